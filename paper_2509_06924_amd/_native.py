"""ctypes binding of the C ABI declared in include/nr.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libnr.so")

NR_OK, NR_EINVAL, NR_EWORKSPACE, NR_EHIP, NR_ENOMEM, NR_ESCRATCH = 0, 1, 2, 3, 4, 5
NR_NOALLOC_SCRATCH_BYTES = 256 << 20
NR_F64, NR_F32 = 0, 1
NR_OP_REFLECTIVITY, NR_OP_LOGLIK, NR_OP_LOGLIK_GRAD = 0, 1, 2
NR_ITEM_NONFINITE, NR_ITEM_BAD_Q, NR_ITEM_BAD_ERR, NR_ITEM_EDGE_SINGULAR = 1, 2, 4, 8
NR_MAX_LAYERS = 40
NR_MAX_DEEP_LAYERS = 2047
NR_SMEAR_NODES = 17
NR_NUM_BUCKETS = 16
NR_VARIANT_AUTO, NR_VARIANT_STORE, NR_VARIANT_RECOMPUTE = 0, 1, 2
NR_TF_FIXED, NR_TF_AFFINE, NR_TF_LOG, NR_TF_LOGIT = 0, 1, 2, 3
NR_HMC_ADAPT_MASS, NR_HMC_ADAPT_STEP = 1, 2
NR_TAILS_LONE, NR_TAILS_SPLIT, NR_SPLIT_SMALL = 1, 2, 4
NR_HMC_MASS_WINDOW_END, NR_HMC_STEP_RESTART, NR_HMC_STEP_FINAL = 1, 2, 4

# every symbol include/nr.h declares
EXPORTS = ("nr_version", "nr_status_string", "nr_plan_create", "nr_plan_destroy",
           "nr_workspace_size", "nr_output_offsets", "nr_reflectivity", "nr_loglik",
           "nr_loglik_grad", "nr_plan_set_timing_events", "nr_leapfrog",
           "nr_leapfrog_graph_create", "nr_graph_launch", "nr_graph_destroy",
           "nr_vi_elbo_grad", "nr_tie_sum", "nr_plan_options_default", "nr_bucket_lmax",
           "nr_store_max_layers", "nr_plan_create_ex", "nr_reflectivity_vjp",
           "nr_loglik_grad_res", "nr_hmc_create", "nr_hmc_destroy", "nr_hmc_init",
           "nr_hmc_transition", "nr_hmc_graph_create", "nr_hmc_adapt", "nr_vi_mvn_create",
           "nr_vi_mvn_destroy", "nr_vi_mvn_step", "nr_vi_mvn_graph_create", "nr_autotune",
           "nr_smearing_rule", "nr_loglik_grad_noalloc")


class BatchDesc(ctypes.Structure):
    _fields_ = [
        ("n_datasets", ctypes.c_int32),
        ("q_off", ctypes.c_void_p),
        ("dq_over_q", ctypes.c_void_p),
        ("n_items", ctypes.c_int32),
        ("dataset_of_item", ctypes.c_void_p),
        ("row_off", ctypes.c_void_p),
        ("precision", ctypes.c_int32),
    ]


class PlanOptions(ctypes.Structure):
    _fields_ = [
        ("grad_variant", ctypes.c_int32 * NR_NUM_BUCKETS),
        ("xcd_run", ctypes.c_int32),
        ("pack_tails", ctypes.c_int32),
        ("split_tails", ctypes.c_int32),
        ("side_stream", ctypes.c_int32),
        ("node_groups", ctypes.c_int32),
    ]


class Values(ctypes.Structure):
    _fields_ = [
        ("q", ctypes.c_void_p),
        ("r_obs", ctypes.c_void_p),
        ("r_err", ctypes.c_void_p),
        ("layers", ctypes.c_void_p),
        ("scale", ctypes.c_void_p),
        ("bkg", ctypes.c_void_p),
        ("item_status", ctypes.c_void_p),
        ("dq", ctypes.c_void_p),
        ("dqq_item", ctypes.c_void_p),
    ]


class HmcState(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in (
        "layers", "scale", "bkg", "mom_rows", "mom_inst", "inv_mass_rows", "inv_mass_inst",
        "logL", "g_rows", "g_inst")]


class HmcConfig(ctypes.Structure):
    _fields_ = [
        ("n_leapfrog", ctypes.c_int32),
        ("max_energy_error", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("target_accept", ctypes.c_double),
    ]


class HmcChains(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in (
        "z_rows", "z_inst", "kind_rows", "kind_inst", "a_rows", "b_rows", "a_inst", "b_inst",
        "inv_mass_rows", "inv_mass_inst", "step", "layers", "scale", "bkg", "logL", "g_rows",
        "g_inst", "potential", "accept_prob", "energy_error", "n_accept", "n_divergent")]


class MvnConfig(ctypes.Structure):
    _fields_ = [
        ("n_restarts", ctypes.c_int32),
        ("n_draws", ctypes.c_int32),
        ("lr", ctypes.c_double),
        ("beta1", ctypes.c_double),
        ("beta2", ctypes.c_double),
        ("adam_eps", ctypes.c_double),
        ("seed", ctypes.c_uint64),
    ]


class MvnParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in (
        "kind", "a", "b", "theta_fixed", "mu", "omega", "lam", "elbo", "grad_mu", "grad_omega",
        "grad_lam")]


class ViArgs(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in (
        "mu", "omega", "mask", "eps", "layers", "scale", "bkg", "logL", "g_rows", "g_inst",
        "grad_mu", "grad_omega", "elbo")]


class NativeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"nr status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libnr.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with python -m paper_2509_06924_amd.build "
                "(the HIP library is the only implementation)")
        # torch ships a HIP runtime of its own under the same soname.  Loading
        # it first makes this library bind to that runtime: one runtime per
        # process, so torch's streams and device pointers are valid here (if
        # this library loaded the system runtime first, torch would then find
        # no GPU).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.nr_version.restype = ctypes.c_int32
        L.nr_status_string.restype = ctypes.c_char_p
        L.nr_status_string.argtypes = [ctypes.c_int32]
        L.nr_plan_create.restype = ctypes.c_int32
        L.nr_plan_create.argtypes = [ctypes.POINTER(BatchDesc), ctypes.POINTER(P)]
        L.nr_plan_create_ex.restype = ctypes.c_int32
        L.nr_plan_create_ex.argtypes = [ctypes.POINTER(BatchDesc), ctypes.POINTER(PlanOptions),
                                        ctypes.POINTER(P)]
        L.nr_plan_options_default.restype = ctypes.c_int32
        L.nr_plan_options_default.argtypes = [ctypes.POINTER(PlanOptions)]
        L.nr_bucket_lmax.restype = ctypes.c_int32
        L.nr_bucket_lmax.argtypes = [ctypes.c_int32]
        L.nr_store_max_layers.restype = ctypes.c_int32
        L.nr_store_max_layers.argtypes = [ctypes.c_int32]
        L.nr_plan_destroy.restype = ctypes.c_int32
        L.nr_plan_destroy.argtypes = [P]
        L.nr_workspace_size.restype = ctypes.c_int32
        L.nr_workspace_size.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
        L.nr_output_offsets.restype = ctypes.c_int32
        L.nr_output_offsets.argtypes = [P, P]
        L.nr_reflectivity.restype = ctypes.c_int32
        L.nr_reflectivity.argtypes = [P, ctypes.POINTER(Values), P, P, ctypes.c_size_t, P]
        L.nr_loglik.restype = ctypes.c_int32
        L.nr_loglik.argtypes = [P, ctypes.POINTER(Values), P, P, ctypes.c_size_t, P]
        L.nr_loglik_grad.restype = ctypes.c_int32
        L.nr_loglik_grad.argtypes = [P, ctypes.POINTER(Values), P, P, P, P, ctypes.c_size_t, P]
        L.nr_loglik_grad_res.restype = ctypes.c_int32
        L.nr_loglik_grad_res.argtypes = [P, ctypes.POINTER(Values), P, P, P, P, P,
                                         ctypes.c_size_t, P]
        L.nr_reflectivity_vjp.restype = ctypes.c_int32
        L.nr_reflectivity_vjp.argtypes = [P, ctypes.POINTER(Values), P, P, P, P, P,
                                          ctypes.c_size_t, P]
        L.nr_plan_set_timing_events.restype = ctypes.c_int32
        L.nr_plan_set_timing_events.argtypes = [P, P, P]
        L.nr_leapfrog.restype = ctypes.c_int32
        L.nr_leapfrog.argtypes = [P, ctypes.POINTER(Values), ctypes.POINTER(HmcState),
                                  ctypes.c_double, ctypes.c_int32, P, ctypes.c_size_t, P]
        L.nr_leapfrog_graph_create.restype = ctypes.c_int32
        L.nr_leapfrog_graph_create.argtypes = [P, ctypes.POINTER(Values), ctypes.POINTER(HmcState),
                                               ctypes.c_double, ctypes.c_int32, P,
                                               ctypes.c_size_t, ctypes.POINTER(P)]
        L.nr_graph_launch.restype = ctypes.c_int32
        L.nr_graph_launch.argtypes = [P, P]
        L.nr_graph_destroy.restype = ctypes.c_int32
        L.nr_graph_destroy.argtypes = [P]
        L.nr_vi_elbo_grad.restype = ctypes.c_int32
        L.nr_vi_elbo_grad.argtypes = [P, ctypes.POINTER(Values), ctypes.POINTER(ViArgs), P,
                                      ctypes.c_size_t, P]
        L.nr_hmc_create.restype = ctypes.c_int32
        L.nr_hmc_create.argtypes = [P, ctypes.POINTER(HmcConfig), ctypes.POINTER(P)]
        L.nr_hmc_destroy.restype = ctypes.c_int32
        L.nr_hmc_destroy.argtypes = [P]
        L.nr_hmc_init.restype = ctypes.c_int32
        L.nr_hmc_init.argtypes = [P, ctypes.POINTER(Values), ctypes.POINTER(HmcChains),
                                  ctypes.c_int32, P, ctypes.c_size_t, P]
        L.nr_hmc_transition.restype = ctypes.c_int32
        L.nr_hmc_transition.argtypes = [P, ctypes.POINTER(Values), ctypes.POINTER(HmcChains),
                                        ctypes.c_int32, P, ctypes.c_size_t, P]
        L.nr_hmc_graph_create.restype = ctypes.c_int32
        L.nr_hmc_graph_create.argtypes = [P, ctypes.POINTER(Values), ctypes.POINTER(HmcChains),
                                          ctypes.c_int32, ctypes.c_int32, P, ctypes.c_size_t,
                                          ctypes.POINTER(P)]
        L.nr_hmc_adapt.restype = ctypes.c_int32
        L.nr_hmc_adapt.argtypes = [P, ctypes.POINTER(HmcChains), ctypes.c_int32, P]
        L.nr_vi_mvn_create.restype = ctypes.c_int32
        L.nr_vi_mvn_create.argtypes = [P, ctypes.POINTER(MvnConfig), ctypes.POINTER(P)]
        L.nr_vi_mvn_destroy.restype = ctypes.c_int32
        L.nr_vi_mvn_destroy.argtypes = [P]
        L.nr_vi_mvn_step.restype = ctypes.c_int32
        L.nr_vi_mvn_step.argtypes = [P, ctypes.POINTER(Values), ctypes.POINTER(MvnParams),
                                     ctypes.c_int32, P, ctypes.c_size_t, P]
        L.nr_vi_mvn_graph_create.restype = ctypes.c_int32
        L.nr_vi_mvn_graph_create.argtypes = [P, ctypes.POINTER(Values), ctypes.POINTER(MvnParams),
                                             ctypes.c_int32, P, ctypes.c_size_t,
                                             ctypes.POINTER(P)]
        L.nr_autotune.restype = ctypes.c_int32
        L.nr_autotune.argtypes = [ctypes.POINTER(BatchDesc), ctypes.POINTER(Values), ctypes.c_int32,
                                  ctypes.POINTER(PlanOptions), P, P]
        L.nr_tie_sum.restype = ctypes.c_int32
        L.nr_tie_sum.argtypes = [ctypes.c_int64, P, P, P, P, P]
        L.nr_loglik_grad_noalloc.restype = ctypes.c_int32
        L.nr_loglik_grad_noalloc.argtypes = [P, ctypes.POINTER(Values), P, P, P, P]
        L.nr_smearing_rule.restype = ctypes.c_int32
        L.nr_smearing_rule.argtypes = [P, P]
        _lib = L
    return _lib


def smearing_rule():
    """The library's quadrature: node offsets t_k (units of sigma_Q) and
    normalised weights w_k, as two lists of NR_SMEAR_NODES floats."""
    t = (ctypes.c_double * NR_SMEAR_NODES)()
    w = (ctypes.c_double * NR_SMEAR_NODES)()
    check(lib().nr_smearing_rule(ctypes.cast(t, ctypes.c_void_p), ctypes.cast(w, ctypes.c_void_p)))
    return list(t), list(w)


def check(status):
    if status != NR_OK:
        raise NativeError(status, lib().nr_status_string(status).decode())
    return status


def status_string(status):
    return lib().nr_status_string(status).decode()
