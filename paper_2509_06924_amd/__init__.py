"""MI355X-native reflectivity log-likelihood and exact gradient (arXiv 2509.06924).

The Python layer only marshals arguments: device memory and streams come from
PyTorch, every step of the computation runs in the HIP library libnr.so
(C ABI in include/nr.h).  There is no CPU fallback: if the library is missing
the calls raise.

    prob = Problem.from_batch(batch, device="cuda")
    logL, g_rows, g_inst = prob.loglik_grad()
    logL = NRLogLik.apply(layers, scale, bkg, prob)   # autograd
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _native as _n
from ._native import (NR_F32, NR_F64, NR_ITEM_BAD_ERR, NR_ITEM_BAD_Q,  # noqa: F401
                      NR_ITEM_EDGE_SINGULAR,
                      NR_ITEM_NONFINITE, NR_MAX_LAYERS, NR_OP_LOGLIK,
                      NR_OP_LOGLIK_GRAD, NR_OP_REFLECTIVITY, NativeError,
                      NR_TF_FIXED, NR_TF_AFFINE, NR_TF_LOG, NR_TF_LOGIT,
                      NR_HMC_ADAPT_MASS, NR_HMC_ADAPT_STEP, NR_HMC_MASS_WINDOW_END,
                      NR_HMC_STEP_RESTART, NR_HMC_STEP_FINAL)

__all__ = ["Plan", "Problem", "plan_options", "bucket_lmax", "NRLogLik", "NRReflectivity",
           "nr_reflectivity", "nr_loglik", "nr_loglik_grad", "pack_theta", "NativeError",
           "HmcState", "LeapfrogGraph", "HMC", "MvnVI", "tie_sum", "tie_map_to_csr"]


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None and a.size else None


def bucket_lmax():
    """Layer-count buckets of the library (deepest layer count of each)."""
    L = _n.lib()
    return [int(L.nr_bucket_lmax(k)) for k in range(_n.NR_NUM_BUCKETS)]


def plan_options(options=None):
    """nr_plan_options from None or a dict (see Plan)."""
    o = _n.PlanOptions()
    _n.check(_n.lib().nr_plan_options_default(ctypes.byref(o)))
    if not options:
        return o
    gv = options.get("grad_variant")
    if gv is not None:
        if isinstance(gv, dict):
            lm = bucket_lmax()
            for key, v in gv.items():
                o.grad_variant[lm.index(int(key))] = int(v)
        else:
            for k, v in enumerate(gv):
                o.grad_variant[k] = int(v)
    if "xcd_run" in options:
        o.xcd_run = int(options["xcd_run"])
    if "pack_tails" in options:
        o.pack_tails = int(options["pack_tails"])
    if "split_tails" in options:
        o.split_tails = int(options["split_tails"])
    if "side_stream" in options:
        o.side_stream = int(options["side_stream"])
    if "node_groups" in options:
        o.node_groups = int(options["node_groups"])
    return o


class Plan:
    """Owns an nr_plan built from host batch structure."""

    def __init__(self, q_off, dq_over_q, dataset_of_item, row_off, precision=NR_F64,
                 options=None):
        """options: None (defaults) or a dict with any of grad_variant (list of
        NR_NUM_BUCKETS ints or {bucket_lmax: variant}), xcd_run, pack_tails,
        split_tails, side_stream, node_groups."""
        self.q_off = np.ascontiguousarray(q_off, np.int64)
        self.dq_over_q = np.ascontiguousarray(dq_over_q, np.float64)
        self.dataset_of_item = np.ascontiguousarray(dataset_of_item, np.int32)
        self.row_off = np.ascontiguousarray(row_off, np.int64)
        d = _n.BatchDesc(self.dq_over_q.size, _ptr(self.q_off), _ptr(self.dq_over_q),
                         self.dataset_of_item.size, _ptr(self.dataset_of_item),
                         _ptr(self.row_off), precision)
        # q_off / row_off are never empty (n+1 entries)
        d.q_off = ctypes.c_void_p(self.q_off.ctypes.data)
        d.row_off = ctypes.c_void_p(self.row_off.ctypes.data)
        h = ctypes.c_void_p()
        self.precision = precision
        self.options = plan_options(options)
        _n.check(_n.lib().nr_plan_create_ex(ctypes.byref(d), ctypes.byref(self.options),
                                            ctypes.byref(h)))
        self._h = h
        self.desc = d  # points into the arrays above, which the plan keeps alive
        self.n_items = int(self.dataset_of_item.size)
        self.n_datasets = int(self.dq_over_q.size)

    @property
    def handle(self):
        return self._h

    def workspace_size(self, op):
        n = ctypes.c_size_t()
        _n.check(_n.lib().nr_workspace_size(self._h, op, ctypes.byref(n)))
        return int(n.value)

    def output_offsets(self):
        out = np.zeros(self.n_items + 1, np.int64)
        _n.check(_n.lib().nr_output_offsets(self._h, ctypes.c_void_p(out.ctypes.data)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            _n.lib().nr_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _values(q, r_obs, r_err, layers, scale, bkg, item_status=None, dq=None, dqq_item=None):
    return _n.Values(_dp(q), _dp(r_obs), _dp(r_err), _dp(layers), _dp(scale), _dp(bkg),
                     _dp(item_status), _dp(dq), _dp(dqq_item))


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def nr_reflectivity(plan, values, r_hat, workspace=None, stream=None):
    ws = _dp(workspace)
    nb = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _n.check(_n.lib().nr_reflectivity(plan.handle, ctypes.byref(values), _dp(r_hat), ws, nb,
                                      _stream(stream)))


def nr_loglik(plan, values, logL, workspace, stream=None):
    nb = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _n.check(_n.lib().nr_loglik(plan.handle, ctypes.byref(values), _dp(logL), _dp(workspace),
                                nb, _stream(stream)))


def nr_loglik_grad(plan, values, logL, g_rows, g_inst, workspace, stream=None):
    nb = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _n.check(_n.lib().nr_loglik_grad(plan.handle, ctypes.byref(values), _dp(logL), _dp(g_rows),
                                     _dp(g_inst), _dp(workspace), nb, _stream(stream)))


def nr_loglik_grad_noalloc(plan, values, logL, g_rows, g_inst, stream=None):
    """nr_loglik_grad on the library's fixed per-GPU scratch (no workspace)."""
    _n.check(_n.lib().nr_loglik_grad_noalloc(plan.handle, ctypes.byref(values), _dp(logL),
                                             _dp(g_rows), _dp(g_inst), _stream(stream)))


class Problem:
    """Datasets resident on the device plus a plan; parameters may be swapped
    per call (same structure)."""

    def __init__(self, plan, q, r_obs, r_err, layers, scale, bkg, device="cuda"):
        import torch
        self.plan = plan
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        f = dict(dtype=torch.float64, device=self.device)
        self.q = torch.as_tensor(q, **f).contiguous()
        self.r_obs = torch.as_tensor(r_obs, **f).contiguous()
        self.r_err = torch.as_tensor(r_err, **f).contiguous()
        self.layers = torch.as_tensor(layers, **f).reshape(-1, 4).contiguous()
        self.scale = torch.as_tensor(scale, **f).contiguous()
        self.bkg = torch.as_tensor(bkg, **f).contiguous()
        self.item_status = torch.zeros(plan.n_items, dtype=torch.int32, device=self.device)
        self.dq = None        # per-point FWHM (packed like q), smeared datasets
        self.dqq_item = None  # per-item relative FWHM dQ/Q
        self._ws = {}
        self.out_off = plan.output_offsets()

    @classmethod
    def from_batch(cls, batch, device="cuda", precision=NR_F64, options=None):
        plan = Plan(batch.q_off, batch.dq_over_q, batch.dataset_of_item, batch.row_off, precision,
                    options)
        return cls(plan, batch.Q, batch.Robs, batch.Rerr, batch.layers, batch.scale, batch.bkg,
                   device)

    def workspace(self, op):
        import torch
        if op not in self._ws:
            n = self.plan.workspace_size(op)
            self._ws[op] = torch.empty(max(1, (n + 7) // 8), dtype=torch.float64,
                                       device=self.device)
        return self._ws[op]

    def set_resolution(self, dq=None, dqq_item=None):
        """Resolution of the smeared datasets (those with dq_over_q > 0):
        per-point FWHM widths `dq` (1/A, packed like q), or a relative width
        dQ/Q per item `dqq_item`; None restores the dataset's dQ/Q."""
        import torch
        f = dict(dtype=torch.float64, device=self.device)
        if dq is not None:
            dq = torch.as_tensor(dq, **f).reshape(-1).contiguous()
            if dq.numel() != self.q.numel():
                raise ValueError("dq must hold one width per data point")
        if dqq_item is not None:
            dqq_item = torch.as_tensor(dqq_item, **f).reshape(-1).contiguous()
            if dqq_item.numel() != self.plan.n_items:
                raise ValueError("dqq_item must hold one value per item")
        self.dq, self.dqq_item = dq, dqq_item
        return self

    def values(self, layers=None, scale=None, bkg=None):
        layers = self.layers if layers is None else layers
        scale = self.scale if scale is None else scale
        bkg = self.bkg if bkg is None else bkg
        for t in (layers, scale, bkg):
            if t.dtype != self.q.dtype or t.device != self.device or not t.is_contiguous():
                raise ValueError("parameters must be contiguous float64 tensors on the device")
        if layers.numel() != self.layers.numel() or scale.numel() != self.plan.n_items \
                or bkg.numel() != self.plan.n_items:
            raise ValueError("parameter sizes do not match the plan")
        return _values(self.q, self.r_obs, self.r_err, layers, scale, bkg, self.item_status,
                       self.dq, self.dqq_item)

    def reflectivity(self, layers=None, scale=None, bkg=None, stream=None):
        import torch
        out = torch.empty(int(self.out_off[-1]), dtype=torch.float64, device=self.device)
        nr_reflectivity(self.plan, self.values(layers, scale, bkg), out,
                        self.workspace(NR_OP_REFLECTIVITY), stream)
        return out

    def loglik(self, layers=None, scale=None, bkg=None, stream=None):
        import torch
        out = torch.empty(self.plan.n_items, dtype=torch.float64, device=self.device)
        nr_loglik(self.plan, self.values(layers, scale, bkg), out,
                  self.workspace(NR_OP_LOGLIK), stream)
        return out

    def loglik_grad(self, layers=None, scale=None, bkg=None, stream=None, out=None):
        import torch
        if out is None:
            out = (torch.empty(self.plan.n_items, dtype=torch.float64, device=self.device),
                   torch.empty_like(self.layers),
                   torch.empty(self.plan.n_items, 2, dtype=torch.float64, device=self.device))
        logL, g_rows, g_inst = out
        nr_loglik_grad(self.plan, self.values(layers, scale, bkg), logL, g_rows, g_inst,
                       self.workspace(NR_OP_LOGLIK_GRAD), stream)
        return logL, g_rows, g_inst

    def loglik_grad_res(self, layers=None, scale=None, bkg=None, stream=None):
        """loglik_grad plus g_res[b] = dlogL_b/d(dQ/Q)_b (0 on unsmeared
        datasets and with per-point widths)."""
        import torch
        logL = torch.empty(self.plan.n_items, dtype=torch.float64, device=self.device)
        g_rows = torch.empty_like(self.layers)
        g_inst = torch.empty(self.plan.n_items, 2, dtype=torch.float64, device=self.device)
        g_res = torch.empty(self.plan.n_items, dtype=torch.float64, device=self.device)
        ws = self.workspace(NR_OP_LOGLIK_GRAD)
        _n.check(_n.lib().nr_loglik_grad_res(
            self.plan.handle, ctypes.byref(self.values(layers, scale, bkg)), _dp(logL),
            _dp(g_rows), _dp(g_inst), _dp(g_res), _dp(ws), ws.numel() * 8, _stream(stream)))
        return logL, g_rows, g_inst, g_res


def _reflectivity_vjp(self, seed, layers=None, scale=None, bkg=None, stream=None):
    """Vector-Jacobian product of R_hat for per-point seeds (packed like
    R_hat): returns (dot = sum_i seed_i R_hat_i per item, g_rows, g_inst)."""
    import torch
    seed_t = torch.as_tensor(seed, dtype=torch.float64, device=self.device).reshape(-1)
    seed_t = seed_t.contiguous()
    if seed_t.numel() != int(self.out_off[-1]):
        raise ValueError("seed must hold one value per data point of every item")
    dot = torch.empty(self.plan.n_items, dtype=torch.float64, device=self.device)
    g_rows = torch.empty_like(self.layers)
    g_inst = torch.empty(self.plan.n_items, 2, dtype=torch.float64, device=self.device)
    ws = self.workspace(NR_OP_LOGLIK_GRAD)
    _n.check(_n.lib().nr_reflectivity_vjp(
        self.plan.handle, ctypes.byref(self.values(layers, scale, bkg)), _dp(seed_t), _dp(dot),
        _dp(g_rows), _dp(g_inst), _dp(ws), ws.numel() * 8, _stream(stream)))
    return dot, g_rows, g_inst


Problem.reflectivity_vjp = _reflectivity_vjp


class HmcState:
    """Device tensors of an HMC state: positions (copies of the problem's
    parameters), momenta, optional inverse masses, and logL/gradient at the
    positions."""

    def __init__(self, problem, mom_rows, mom_inst, inv_mass_rows=None, inv_mass_inst=None):
        import torch
        f = dict(dtype=torch.float64, device=problem.device)
        self.layers = problem.layers.clone()
        self.scale = problem.scale.clone()
        self.bkg = problem.bkg.clone()
        self.mom_rows = torch.as_tensor(mom_rows, **f).reshape(-1, 4).contiguous().clone()
        self.mom_inst = torch.as_tensor(mom_inst, **f).reshape(-1, 2).contiguous().clone()
        self.inv_mass_rows = None if inv_mass_rows is None else \
            torch.as_tensor(inv_mass_rows, **f).reshape(-1, 4).contiguous()
        self.inv_mass_inst = None if inv_mass_inst is None else \
            torch.as_tensor(inv_mass_inst, **f).reshape(-1, 2).contiguous()
        self.logL, self.g_rows, self.g_inst = problem.loglik_grad(
            self.layers, self.scale, self.bkg)

    def native(self):
        return _n.HmcState(*[_dp(t) for t in (
            self.layers, self.scale, self.bkg, self.mom_rows, self.mom_inst, self.inv_mass_rows,
            self.inv_mass_inst, self.logL, self.g_rows, self.g_inst)])


class LeapfrogGraph:
    """n leapfrog steps captured once in a HIP graph; launch() replays them."""

    def __init__(self, problem, state, dt, n_steps):
        self._problem, self._state = problem, state  # keep pointers alive
        self._data = problem.values()
        self._st = state.native()
        ws = problem.workspace(NR_OP_LOGLIK_GRAD)
        h = ctypes.c_void_p()
        _n.check(_n.lib().nr_leapfrog_graph_create(
            problem.plan.handle, ctypes.byref(self._data), ctypes.byref(self._st), dt, n_steps,
            _dp(ws), ws.numel() * 8, ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _n.check(_n.lib().nr_graph_launch(self._h, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None):
            _n.lib().nr_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Graph:
    """A captured HIP graph (nr_graph); launch() replays it."""

    def __init__(self, handle, keep):
        self._h = handle
        self._keep = keep  # objects whose device pointers the graph holds

    def launch(self, stream=None):
        _n.check(_n.lib().nr_graph_launch(self._h, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None):
            _n.lib().nr_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class HMC:
    """HMC driver (nr_hmc_*): the problem's items are independent chains.

    Per entry (rows as (R, 4), instrument as (n, 2) [scale, bkg]): the
    transform kind (NR_TF_*), its constants a and b, and the diagonal inverse
    mass; per chain the leapfrog step.  The chain starts at the problem's
    parameters (z from theta on init).  Device tensors after each call:
    z_rows/z_inst, layers/scale/bkg (theta), logL, g_rows, g_inst, potential,
    accept_prob, energy_error, n_accept, n_divergent, inv_mass_*, step."""

    def __init__(self, problem, kind_rows=None, kind_inst=None, a_rows=None, b_rows=None,
                 a_inst=None, b_inst=None, inv_mass_rows=None, inv_mass_inst=None, step=0.01,
                 n_leapfrog=10, max_energy_error=1000.0, seed=0, target_accept=0.8):
        import torch
        self.problem = problem
        dev = problem.device
        n = problem.plan.n_items
        R = problem.layers.shape[0]
        f = dict(dtype=torch.float64, device=dev)

        def arr(v, shape, default, dtype=torch.float64):
            if v is None:
                return torch.full(shape, default, dtype=dtype, device=dev)
            return torch.as_tensor(v, dtype=dtype, device=dev).reshape(shape).contiguous().clone()

        self.kind_rows = arr(kind_rows, (R, 4), NR_TF_AFFINE, torch.uint8)
        self.kind_inst = arr(kind_inst, (n, 2), NR_TF_AFFINE, torch.uint8)
        self.a_rows = arr(a_rows, (R, 4), 0.0)
        self.b_rows = arr(b_rows, (R, 4), 1.0)
        self.a_inst = arr(a_inst, (n, 2), 0.0)
        self.b_inst = arr(b_inst, (n, 2), 1.0)
        self.inv_mass_rows = arr(inv_mass_rows, (R, 4), 1.0)
        self.inv_mass_inst = arr(inv_mass_inst, (n, 2), 1.0)
        self.step = (torch.full((n,), float(step), **f) if np.ndim(step) == 0
                     else arr(step, (n,), 0.0))
        self.layers = problem.layers.clone()
        self.scale = problem.scale.clone()
        self.bkg = problem.bkg.clone()
        self.z_rows = torch.zeros(R, 4, **f)
        self.z_inst = torch.zeros(n, 2, **f)
        self.logL = torch.zeros(n, **f)
        self.g_rows = torch.zeros(R, 4, **f)
        self.g_inst = torch.zeros(n, 2, **f)
        self.potential = torch.zeros(n, **f)
        self.accept_prob = torch.zeros(n, **f)
        self.energy_error = torch.zeros(n, **f)
        self.n_accept = torch.zeros(n, dtype=torch.int32, device=dev)
        self.n_divergent = torch.zeros(n, dtype=torch.int32, device=dev)
        self.config = _n.HmcConfig(int(n_leapfrog), float(max_energy_error), int(seed),
                                   float(target_accept))
        h = ctypes.c_void_p()
        _n.check(_n.lib().nr_hmc_create(problem.plan.handle, ctypes.byref(self.config),
                                        ctypes.byref(h)))
        self._h = h
        self._chains = _n.HmcChains(*[_dp(t) for t in (
            self.z_rows, self.z_inst, self.kind_rows, self.kind_inst, self.a_rows, self.b_rows,
            self.a_inst, self.b_inst, self.inv_mass_rows, self.inv_mass_inst, self.step,
            self.layers, self.scale, self.bkg, self.logL, self.g_rows, self.g_inst,
            self.potential, self.accept_prob, self.energy_error, self.n_accept,
            self.n_divergent)])
        self._data = problem.values()

    def _ws(self):
        ws = self.problem.workspace(NR_OP_LOGLIK_GRAD)
        return _dp(ws), ws.numel() * 8

    def init(self, from_theta=True, stream=None):
        ws, nb = self._ws()
        _n.check(_n.lib().nr_hmc_init(self._h, ctypes.byref(self._data),
                                      ctypes.byref(self._chains), int(bool(from_theta)), ws, nb,
                                      _stream(stream)))
        return self

    @staticmethod
    def _adapt_bits(adapt_mass, adapt_step):
        return (NR_HMC_ADAPT_MASS if adapt_mass else 0) | (NR_HMC_ADAPT_STEP if adapt_step else 0)

    def transition(self, adapt_mass=False, adapt_step=False, stream=None):
        ws, nb = self._ws()
        _n.check(_n.lib().nr_hmc_transition(self._h, ctypes.byref(self._data),
                                            ctypes.byref(self._chains),
                                            self._adapt_bits(adapt_mass, adapt_step), ws, nb,
                                            _stream(stream)))

    def graph(self, n_transitions=1, adapt_mass=False, adapt_step=False):
        ws, nb = self._ws()
        g = ctypes.c_void_p()
        _n.check(_n.lib().nr_hmc_graph_create(self._h, ctypes.byref(self._data),
                                              ctypes.byref(self._chains),
                                              self._adapt_bits(adapt_mass, adapt_step),
                                              int(n_transitions), ws, nb, ctypes.byref(g)))
        return _Graph(g, self)

    def adapt(self, mass_window_end=False, step_restart=False, step_final=False, stream=None):
        bits = ((NR_HMC_MASS_WINDOW_END if mass_window_end else 0)
                | (NR_HMC_STEP_RESTART if step_restart else 0)
                | (NR_HMC_STEP_FINAL if step_final else 0))
        _n.check(_n.lib().nr_hmc_adapt(self._h, ctypes.byref(self._chains), bits,
                                       _stream(stream)))

    def close(self):
        if getattr(self, "_h", None):
            _n.lib().nr_hmc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MvnVI:
    """Full-rank Gaussian VI driver (nr_vi_mvn_*): `problem` has R x S items
    (restart r, draw s at item r S + s) with equal rows.  Per entry (P =
    4 rows + 2: the rows, then scale, bkg) the transform kind and constants
    and the value of entries that do not move; per restart mu (default from
    the inverse transform of theta_fixed), omega = softplus^-1(sigma0) and
    lambda = 0.  Device tensors: mu (R, P), omega (R, P), lam (R, P, P),
    elbo (R,), grad_mu, grad_omega, grad_lam."""

    def __init__(self, problem, n_restarts, n_draws, kind, a, b, theta_fixed, mu=None,
                 sigma0=0.1, lr=0.05, beta1=0.9, beta2=0.999, adam_eps=1e-8, seed=0):
        import torch
        dev = problem.device
        f = dict(dtype=torch.float64, device=dev)
        R, S = int(n_restarts), int(n_draws)
        self.problem = problem
        self.kind = torch.as_tensor(kind, dtype=torch.uint8, device=dev).reshape(-1).contiguous()
        P = self.kind.numel()
        self.a = torch.as_tensor(a, **f).reshape(P).contiguous()
        self.b = torch.as_tensor(b, **f).reshape(P).contiguous()
        self.theta_fixed = torch.as_tensor(theta_fixed, **f).reshape(P).contiguous()
        if mu is None:
            raise ValueError("mu (R x P, unconstrained) is required")
        self.mu = torch.as_tensor(mu, **f).reshape(R, P).contiguous().clone()
        w = float(sigma0 + np.log(-np.expm1(-sigma0)))
        self.omega = torch.full((R, P), w, **f)
        self.lam = torch.zeros(R, P, P, **f)
        self.elbo = torch.zeros(R, **f)
        self.grad_mu = torch.zeros(R, P, **f)
        self.grad_omega = torch.zeros(R, P, **f)
        self.grad_lam = torch.zeros(R, P, P, **f)
        self.config = _n.MvnConfig(R, S, float(lr), float(beta1), float(beta2), float(adam_eps),
                                   int(seed))
        h = ctypes.c_void_p()
        _n.check(_n.lib().nr_vi_mvn_create(problem.plan.handle, ctypes.byref(self.config),
                                           ctypes.byref(h)))
        self._h = h
        self._prm = _n.MvnParams(*[_dp(t) for t in (
            self.kind, self.a, self.b, self.theta_fixed, self.mu, self.omega, self.lam,
            self.elbo, self.grad_mu, self.grad_omega, self.grad_lam)])
        self._data = problem.values()

    def _ws(self):
        ws = self.problem.workspace(NR_OP_LOGLIK_GRAD)
        return _dp(ws), ws.numel() * 8

    def step(self, adam=True, stream=None):
        ws, nb = self._ws()
        _n.check(_n.lib().nr_vi_mvn_step(self._h, ctypes.byref(self._data),
                                         ctypes.byref(self._prm), int(bool(adam)), ws, nb,
                                         _stream(stream)))

    def graph(self, n_steps=1):
        ws, nb = self._ws()
        g = ctypes.c_void_p()
        _n.check(_n.lib().nr_vi_mvn_graph_create(self._h, ctypes.byref(self._data),
                                                 ctypes.byref(self._prm), int(n_steps), ws, nb,
                                                 ctypes.byref(g)))
        return _Graph(g, self)

    def close(self):
        if getattr(self, "_h", None):
            _n.lib().nr_vi_mvn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _leapfrog(self, state, dt, n_steps, stream=None):
    ws = self.workspace(NR_OP_LOGLIK_GRAD)
    data = self.values()
    st = state.native()
    _n.check(_n.lib().nr_leapfrog(self.plan.handle, ctypes.byref(data), ctypes.byref(st), dt,
                                  n_steps, _dp(ws), ws.numel() * 8, _stream(stream)))


def _vi_elbo_grad(self, mu, omega, mask, eps, stream=None):
    """ELBO estimate and its gradient w.r.t. (mu, omega); returns
    (elbo, grad_mu, grad_omega, logL per sample)."""
    import torch
    dev = self.device
    P = int(np.asarray(mu).size) if not hasattr(mu, "numel") else int(mu.numel())
    f = dict(dtype=torch.float64, device=dev)
    mu_t = torch.as_tensor(mu, **f).reshape(-1).contiguous()
    om_t = torch.as_tensor(omega, **f).reshape(-1).contiguous()
    mask_t = torch.as_tensor(mask, dtype=torch.uint8, device=dev).reshape(-1).contiguous()
    eps_t = torch.as_tensor(eps, **f).reshape(-1).contiguous()
    S = self.plan.n_items
    if eps_t.numel() != S * P:
        raise ValueError("eps must hold n_items x P draws")
    out = dict(layers=torch.empty_like(self.layers), scale=torch.empty(S, **f),
               bkg=torch.empty(S, **f), logL=torch.empty(S, **f),
               g_rows=torch.empty_like(self.layers), g_inst=torch.empty(S, 2, **f),
               grad_mu=torch.empty(P, **f), grad_omega=torch.empty(P, **f),
               elbo=torch.empty(1, **f))
    args = _n.ViArgs(_dp(mu_t), _dp(om_t), _dp(mask_t), _dp(eps_t), *[_dp(out[k]) for k in (
        "layers", "scale", "bkg", "logL", "g_rows", "g_inst", "grad_mu", "grad_omega", "elbo")])
    ws = self.workspace(NR_OP_LOGLIK_GRAD)
    data = self.values()
    _n.check(_n.lib().nr_vi_elbo_grad(self.plan.handle, ctypes.byref(data), ctypes.byref(args),
                                      _dp(ws), ws.numel() * 8, _stream(stream)))
    return out["elbo"], out["grad_mu"], out["grad_omega"], out["logL"]


Problem.leapfrog = _leapfrog
Problem.vi_elbo_grad = _vi_elbo_grad


def tie_sum(first, src, values, stream=None):
    """out[k] = sum_{t in [first[k], first[k+1])} values[src[t]] on the device."""
    import torch
    dev = values.device
    first_t = torch.as_tensor(first, dtype=torch.int64, device=dev).contiguous()
    src_t = torch.as_tensor(src, dtype=torch.int64, device=dev).contiguous()
    vals = values.contiguous().reshape(-1)
    out = torch.empty(first_t.numel() - 1, dtype=torch.float64, device=dev)
    _n.check(_n.lib().nr_tie_sum(out.numel(), _dp(first_t), _dp(src_t), _dp(vals), _dp(out),
                                 _stream(stream)))
    return out


def tie_map_to_csr(tie_of_entry, n_out):
    """CSR (first, src) from an array giving, for every source entry, the
    shared parameter it belongs to (or -1)."""
    tie = np.asarray(tie_of_entry, np.int64).reshape(-1)
    src = np.nonzero(tie >= 0)[0]
    order = np.argsort(tie[src], kind="stable")
    src = src[order]
    counts = np.bincount(tie[src], minlength=n_out)
    first = np.zeros(n_out + 1, np.int64)
    first[1:] = np.cumsum(counts)
    return first, src.astype(np.int64)


def _make_autograd():
    import torch

    class NRLogLik(torch.autograd.Function):
        """logL per item as a differentiable function of (layers, scale, bkg).

        Forward runs the fused value+gradient kernel when any input needs a
        gradient and keeps the gradient; backward scales it by grad_output."""

        @staticmethod
        def forward(ctx, layers, scale, bkg, problem):
            need = any(ctx.needs_input_grad[:3])
            if need:
                logL, g_rows, g_inst = problem.loglik_grad(layers.detach().contiguous(),
                                                           scale.detach().contiguous(),
                                                           bkg.detach().contiguous())
                ctx.save_for_backward(g_rows, g_inst)
                ctx.row_item = problem.row_item
            else:
                logL = problem.loglik(layers.detach().contiguous(), scale.detach().contiguous(),
                                      bkg.detach().contiguous())
            return logL

        @staticmethod
        def backward(ctx, grad_out):
            g_rows, g_inst = ctx.saved_tensors
            go_rows = grad_out[ctx.row_item].unsqueeze(1)
            return g_rows * go_rows, g_inst[:, 0] * grad_out, g_inst[:, 1] * grad_out, None

    class NRReflectivity(torch.autograd.Function):
        """R_hat (packed item-major, nr_output_offsets) as a differentiable
        function of (layers, scale, bkg); backward is nr_reflectivity_vjp."""

        @staticmethod
        def forward(ctx, layers, scale, bkg, problem):
            args = [t.detach().contiguous() for t in (layers, scale, bkg)]
            ctx.problem = problem
            ctx.save_for_backward(*args)
            return problem.reflectivity(*args)

        @staticmethod
        def backward(ctx, grad_out):
            layers, scale, bkg = ctx.saved_tensors
            _, g_rows, g_inst = ctx.problem.reflectivity_vjp(grad_out.contiguous(), layers,
                                                              scale, bkg)
            return g_rows, g_inst[:, 0], g_inst[:, 1], None

    return NRLogLik, NRReflectivity


class _LazyAutograd:
    _cls = None

    def __init__(self, which):
        self._which = which

    def __getattr__(self, name):
        if _LazyAutograd._cls is None:
            _LazyAutograd._cls = _make_autograd()
        return getattr(_LazyAutograd._cls[self._which], name)


NRLogLik = _LazyAutograd(0)
NRReflectivity = _LazyAutograd(1)


def _row_item(problem):
    import torch
    ro = problem.plan.row_off
    idx = np.repeat(np.arange(problem.plan.n_items), np.diff(ro))
    return torch.as_tensor(idx, dtype=torch.int64, device=problem.device)


Problem.row_item = property(lambda self: self.__dict__.setdefault("_row_item", _row_item(self)))


def pack_theta(theta, sld_unit=1.0):
    """Rows [d, rho_re, rho_im, sigma] from the paper's parameter dict
    (Sec. 3): thick (n,), SLD (n+2,), rough (n+1,), optional iSLD (n+2,).
    sld_unit multiplies SLD values (1e-6 for values given in 1e-6 A^-2)."""
    thick = np.atleast_1d(np.asarray(theta["thick"], np.float64))
    sld = np.atleast_1d(np.asarray(theta["SLD"], np.float64)) * sld_unit
    rough = np.atleast_1d(np.asarray(theta["rough"], np.float64))
    n = thick.size
    if sld.size != n + 2 or rough.size != n + 1:
        raise ValueError("expected thick (n,), SLD (n+2,), rough (n+1,)")
    rows = np.zeros((n + 2, 4))
    rows[1:n + 1, 0] = thick
    rows[:, 1] = sld
    if "iSLD" in theta:
        rows[:, 2] = np.asarray(theta["iSLD"], np.float64) * sld_unit
    rows[1:, 3] = rough
    return rows
