"""Register, scratch, LDS and occupancy budget of the gradient kernels, as the
compiler reports it (-Rpass-analysis=kernel-resource-usage, device-only
compiles of the kernel sources with the library's flags).  The speed of the
layer-product kernels rests on these figures (waves per SIMD, no spill where
none is expected); a compiler or source change that moves them fails here
instead of showing up only as a slower benchmark."""
import os
import re
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2509_06924_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# (translation unit, defines) -> kernels checked in it.  Kernel key:
# (precision, LMAX, store, tail, res, split) of k_loglik_grad, or
# ("scan", levels per lane, waves, res) of k_loglik_grad_scan.
# Expected: (VGPRs, AGPRs, scratch bytes per lane, waves per SIMD, LDS bytes).
BUDGET = {
    ("nr_kernels_f64.hip", ()): {
        ("F64", 4, 1, 0, 0, 0): (237, 0, 0, 2, 18192),
        ("F64", 10, 1, 0, 0, 0): (256, 232, 0, 1, 36624),
        ("F64", 10, 0, 0, 0, 0): (255, 0, 12, 2, 20240),
        ("F64", 10, 0, 0, 1, 0): (245, 0, 0, 2, 20240),
        ("F64", 10, 0, 0, 0, 1): (254, 0, 20, 2, 20240),
        ("F64", 12, 0, 0, 0, 0): (247, 0, 0, 2, 20240),
    },
    ("nr_kernels_bucket.hip", ("F64", 14)): {
        ("F64", 14, 0, 0, 0, 0): (255, 0, 60, 2, 20240),
    },
    ("nr_kernels_bucket.hip", ("F64", 24)): {
        ("F64", 24, 0, 0, 0, 0): (256, 224, 0, 1, 40720),
    },
    ("nr_kernels_bucket.hip", ("F64", 40)): {
        ("F64", 40, 0, 0, 0, 0): (256, 256, 400, 1, 40720),
    },
    ("nr_kernels_f32.hip", ()): {
        ("F32", 8, 1, 0, 0, 0): (239, 0, 0, 2, 16656),
        ("F32", 10, 0, 0, 0, 0): (167, 0, 0, 3, 12048),
    },
    ("nr_kernels_bucket.hip", ("F32", 20)): {
        ("F32", 20, 0, 0, 0, 0): (256, 0, 68, 2, 20240),
    },
    ("nr_kernels_bucket.hip", ("F32", 24)): {
        ("F32", 24, 0, 0, 0, 0): (256, 0, 228, 2, 20240),
    },
    ("nr_kernels_bucket.hip", ("F32", 40)): {
        ("F32", 40, 0, 0, 0, 0): (256, 220, 0, 1, 40720),
    },
    ("nr_kernels_scan.hip", ()): {
        ("scan", 8, 1, 0): (253, 0, 0, 2, 19216),
        ("scan", 8, 2, 0): (254, 0, 0, 2, 35808),
        ("scan", 8, 4, 0): (256, 0, 132, 2, 68784),
    },
}


def _mangled(key):
    if key[0] == "scan":
        _, ch, nw, res = key
        return f"_ZN2nr18k_loglik_grad_scanILi{ch}ELi{nw}ELb{res}EEEvNS_10KernelArgsE"
    p, lm, st, tail, res, split = key
    return (f"_ZN2nr13k_loglik_gradINS_3{p}ELi{lm}ELb{st}ELb{tail}ELb{res}ELb{split}EE"
            "EvNS_10KernelArgsE")


def _flags(src):
    import sys
    sys.path.insert(0, ROOT)
    from paper_2509_06924_amd import build
    return [f for f in build.FLAGS if f != "-fPIC"] + build.tu_flags(src)


def _remarks(job, tmp):
    src, defs = job
    d = [] if not defs else [f"-DNR_PREC={defs[0]}", f"-DNR_BUCKET_LMAX={defs[1]}"]
    out = os.path.join(tmp, os.path.basename(src) + "".join(map(str, defs)) + ".o")
    cmd = [HIPCC, *_flags(src), *d, "--cuda-device-only", "-c", os.path.join(CSRC, src), "-o", out,
           "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    res, cur = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"remark: Function Name: (\S+)", line)
        if m:
            cur = res.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+(.+?): (\S+) \[-Rpass-analysis", line)
        if m and cur is not None:
            cur[m.group(1).strip()] = m.group(2)
    return res


@pytest.mark.slow
def test_kernel_register_scratch_lds_budget(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    jobs = list(BUDGET)
    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 4)) as ex:
        found = list(ex.map(lambda j: _remarks(j, str(tmp_path)), jobs))
    bad = []
    for job, rem in zip(jobs, found):
        for key, want in BUDGET[job].items():
            r = rem.get(_mangled(key))
            assert r is not None, f"{key} not compiled in {job}"
            got = (int(r["VGPRs"]), int(r["AGPRs"]), int(r["ScratchSize [bytes/lane]"]),
                   int(r["Occupancy [waves/SIMD]"]), int(r["LDS Size [bytes/block]"]))
            if got != want:
                bad.append(f"{key}: (VGPR, AGPR, scratch, waves, LDS) = {got}, expected {want}")
    assert not bad, "\n".join(bad)
