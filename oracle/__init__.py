"""Plain FP64 CPU oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never does.  It loads
``liborc.so`` built from ``nr_oracle.cpp`` (which states what it computes, the
paper passages it follows and what pins each function) and exposes NumPy-level
wrappers.  Rows are arrays of shape (L+2, 4): [d, rho_re, rho_im, sigma].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nr_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liborc.so")
_lib = None

_D = ctypes.c_double
_I = ctypes.c_int
_P = ctypes.c_void_p


def build() -> str:
    """Compile liborc.so with g++ (no FMA contraction, OpenMP over items)."""
    tmp = _LIB_PATH + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fopenmp",
           "-shared", "-fPIC", "-o", tmp, _SRC]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = ctypes.CDLL(_LIB_PATH)
        _lib.orc_loglik.restype = _D
    return _lib


def _p(a):
    return a.ctypes.data_as(_P)


def _rows(rows):
    r = np.ascontiguousarray(rows, dtype=np.float64)
    assert r.ndim == 2 and r.shape[1] == 4 and r.shape[0] >= 2
    return r, r.shape[0] - 2


def _vec(x):
    return np.ascontiguousarray(np.atleast_1d(np.asarray(x, dtype=np.float64)))


def _check(rc):
    if rc < 0:
        raise ValueError("oracle rejected its arguments")
    return rc


def gauss_legendre17():
    x = np.empty(17)
    u = np.empty(17)
    lib().orc_gauss_legendre17(_p(x), _p(u))
    return x, u


def smear_rule(dq_over_q):
    t = np.empty(17)
    w = np.empty(17)
    K = _check(lib().orc_smear_rule(_D(dq_over_q), _p(t), _p(w)))
    return t[:K].copy(), w[:K].copy()


def smear_nodes(Q, dq_over_q):
    Q = _vec(Q)
    out = np.empty(Q.size * 17)
    K = _check(lib().orc_smear_nodes(_I(Q.size), _p(Q), _D(dq_over_q), _p(out)))
    return out[: Q.size * K].reshape(Q.size, K)


def kz(x, y):
    out = np.empty(2)
    lib().orc_kz(_D(x), _D(y), _p(out))
    return complex(out[0], out[1])


def reflectivity(rows, q):
    r, L = _rows(rows)
    q = _vec(q)
    R = np.empty(q.size)
    _check(lib().orc_reflectivity(_I(L), _p(r), _I(q.size), _p(q), _p(R)))
    return R


def reflectivity_parratt(rows, q):
    r, L = _rows(rows)
    q = _vec(q)
    R = np.empty(q.size)
    _check(lib().orc_reflectivity_parratt(_I(L), _p(r), _I(q.size), _p(q), _p(R)))
    return R


def reflectivity_linsys(rows, q):
    r, L = _rows(rows)
    q = _vec(q)
    R = np.empty(q.size)
    _check(lib().orc_reflectivity_linsys(_I(L), _p(r), _I(q.size), _p(q), _p(R)))
    return R


def model_curve(rows, scale, bkg, Q, dq_over_q):
    r, L = _rows(rows)
    Q = _vec(Q)
    out = np.empty(Q.size)
    _check(lib().orc_model_curve(_I(L), _p(r), _D(scale), _D(bkg), _I(Q.size),
                                 _p(Q), _D(dq_over_q), _p(out)))
    return out


def smeared(rows, Q, dq_over_q):
    r, L = _rows(rows)
    Q = _vec(Q)
    out = np.empty(Q.size)
    _check(lib().orc_smeared(_I(L), _p(r), _I(Q.size), _p(Q), _D(dq_over_q), _p(out)))
    return out


def loglik(rows, scale, bkg, Q, Robs, Rerr, dq_over_q):
    r, L = _rows(rows)
    Q, Robs, Rerr = _vec(Q), _vec(Robs), _vec(Rerr)
    return lib().orc_loglik(_I(L), _p(r), _D(scale), _D(bkg), _I(Q.size), _p(Q),
                            _p(Robs), _p(Rerr), _D(dq_over_q))


def loglik_grad_cs(rows, scale, bkg, Q, Robs, Rerr, dq_over_q):
    """logL, gradient rows (L+2, 4), and [d/dscale, d/dbkg] by complex step."""
    r, L = _rows(rows)
    Q, Robs, Rerr = _vec(Q), _vec(Robs), _vec(Rerr)
    ll = np.empty(1)
    g = np.empty_like(r)
    gi = np.empty(2)
    _check(lib().orc_loglik_grad_cs(_I(L), _p(r), _D(scale), _D(bkg), _I(Q.size),
                                    _p(Q), _p(Robs), _p(Rerr), _D(dq_over_q),
                                    _p(ll), _p(g), _p(gi)))
    return ll[0], g, gi


def loglik_grad_fd(rows, scale, bkg, Q, Robs, Rerr, dq_over_q, rel_step=1e-3):
    r, L = _rows(rows)
    Q, Robs, Rerr = _vec(Q), _vec(Robs), _vec(Rerr)
    g = np.empty_like(r)
    gi = np.empty(2)
    _check(lib().orc_loglik_grad_fd(_I(L), _p(r), _D(scale), _D(bkg), _I(Q.size),
                                    _p(Q), _p(Robs), _p(Rerr), _D(dq_over_q),
                                    _D(rel_step), _p(g), _p(gi)))
    return g, gi


def model_vjp_cs(rows, scale, bkg, Q, dq_over_q, seed):
    r, L = _rows(rows)
    Q, seed = _vec(Q), _vec(seed)
    g = np.empty_like(r)
    gi = np.empty(2)
    _check(lib().orc_model_vjp_cs(_I(L), _p(r), _D(scale), _D(bkg), _I(Q.size),
                                  _p(Q), _D(dq_over_q), _p(seed), _p(g), _p(gi)))
    return g, gi


def reflectivity_jac_cs(rows, q):
    """dR(q_i)/d rows, shape (nq, L+2, 4)."""
    r, L = _rows(rows)
    q = _vec(q)
    out = np.empty((q.size, L + 2, 4))
    _check(lib().orc_reflectivity_jac_cs(_I(L), _p(r), _I(q.size), _p(q), _p(out)))
    return out


def loglik_grad_batch(q_off, Q, Robs, Rerr, dq_over_q, dataset_of_item, row_off,
                      layers, scale, bkg, want_grad=True, nthreads=1):
    """Batched logL (and gradient) over items; arrays as in the C ABI."""
    q_off = np.ascontiguousarray(q_off, dtype=np.int64)
    row_off = np.ascontiguousarray(row_off, dtype=np.int64)
    dsi = np.ascontiguousarray(dataset_of_item, dtype=np.int32)
    Q, Robs, Rerr = _vec(Q), _vec(Robs), _vec(Rerr)
    dqq = _vec(dq_over_q)
    layers = np.ascontiguousarray(layers, dtype=np.float64).reshape(-1)
    scale, bkg = _vec(scale), _vec(bkg)
    n_items = dsi.size
    ll = np.empty(n_items)
    g = np.zeros_like(layers)
    gi = np.zeros(2 * n_items)
    _check(lib().orc_loglik_grad_batch(
        _I(q_off.size - 1), _p(q_off), _p(Q), _p(Robs), _p(Rerr), _p(dqq),
        _I(n_items), _p(dsi), _p(row_off), _p(layers), _p(scale), _p(bkg),
        _I(1 if want_grad else 0), _I(nthreads), _p(ll), _p(g), _p(gi)))
    return ll, g, gi.reshape(n_items, 2)


def reflectivity_dq_cs(rows, q):
    """dR/dq of the unsmeared R (complex step through q)."""
    r, L = _rows(rows)
    q = _vec(q)
    out = np.empty_like(q)
    _check(lib().orc_reflectivity_dq_cs(_I(L), _p(r), _I(q.size), _p(q), _p(out)))
    return out


def model_curve_res(rows, scale, bkg, Q, dq_over_q, dQ=None):
    """R_hat with per-point FWHMs dQ (None: dq_over_q * Q)."""
    r, L = _rows(rows)
    Q = _vec(Q)
    out = np.empty_like(Q)
    dq = None if dQ is None else _vec(dQ)
    _check(lib().orc_model_curve_res(_I(L), _p(r), _D(scale), _D(bkg), _I(Q.size), _p(Q),
                                     _D(dq_over_q), None if dq is None else _p(dq), _p(out)))
    return out


def loglik_grad_res_cs(rows, scale, bkg, Q, Robs, Rerr, dq_over_q, dQ=None):
    """(logL, g_rows, g_inst, dlogL/d(dQ/Q)) by complex step; per-point FWHMs
    dQ are data (their derivative is not taken; g_res is then 0)."""
    r, L = _rows(rows)
    Q, Robs, Rerr = _vec(Q), _vec(Robs), _vec(Rerr)
    dq = None if dQ is None else _vec(dQ)
    ll = ctypes.c_double()
    gr = ctypes.c_double()
    g = np.zeros_like(r)
    gi = np.zeros(2)
    _check(lib().orc_loglik_grad_res_cs(
        _I(L), _p(r), _D(scale), _D(bkg), _I(Q.size), _p(Q), _p(Robs), _p(Rerr),
        _D(dq_over_q), None if dq is None else _p(dq), ctypes.byref(ll), _p(g), _p(gi),
        ctypes.byref(gr)))
    return ll.value, g, gi, gr.value


def loglik_res_fd(rows, scale, bkg, Q, Robs, Rerr, dq_over_q, rel_step=1e-3):
    """Richardson difference of logL in dQ/Q."""
    r, L = _rows(rows)
    Q, Robs, Rerr = _vec(Q), _vec(Robs), _vec(Rerr)
    gr = ctypes.c_double()
    _check(lib().orc_loglik_res_fd(_I(L), _p(r), _D(scale), _D(bkg), _I(Q.size), _p(Q),
                                   _p(Robs), _p(Rerr), _D(dq_over_q), _D(rel_step),
                                   ctypes.byref(gr)))
    return gr.value


def max_threads():
    return lib().orc_max_threads()
