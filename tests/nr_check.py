"""Comparison helpers shared by the parity tests (tolerances from the task's
accuracy targets: 1e-10 relative in R, 1e-8 in the gradient; the logL bound is
propagated from the R bound through the likelihood)."""
import numpy as np

R_TOL = 1e-10
G_TOL = 1e-8
# natural units for gradient scaling: d, sigma in A; rho in 1e-6 A^-2
ROW_UNITS = np.array([1.0, 1e-6, 1e-6, 1.0])
INST_UNITS = np.array([1.0, 1e-7])


def check_R(R_k, R_o, tol=R_TOL, what="R"):
    R_k = np.asarray(R_k, float)
    R_o = np.asarray(R_o, float)
    assert R_k.shape == R_o.shape, (R_k.shape, R_o.shape)
    if R_o.size == 0:
        return 0.0
    err = np.abs(R_k - R_o) / np.abs(R_o)
    worst = float(np.max(err))
    assert worst <= tol, f"{what}: max rel err {worst:.3e} at {int(np.argmax(err))}"
    return worst


def logL_bound(Rhat, Robs, Rerr, tol=R_TOL):
    """|d logL| <= sum_i |z_i| / e_i * tol * |R_hat_i| (first order in the R error)."""
    z = (Rhat - Robs) / Rerr
    return float(np.sum(np.abs(z) / Rerr * tol * np.abs(Rhat))) + 1e-13 * float(np.sum(0.5 * z * z + np.abs(np.log(Rerr))) + 1.0)


def check_logL(ll_k, ll_o, bound, what="logL"):
    d = abs(float(ll_k) - float(ll_o))
    assert d <= bound, f"{what}: |diff| {d:.3e} > bound {bound:.3e} (ref {ll_o:.6e})"
    return d


def check_grad(g_rows_k, g_inst_k, g_rows_o, g_inst_o, tol=G_TOL, what="grad"):
    a = np.concatenate([(np.asarray(g_rows_k) * ROW_UNITS).ravel(),
                        np.asarray(g_inst_k).ravel() * INST_UNITS])
    b = np.concatenate([(np.asarray(g_rows_o) * ROW_UNITS).ravel(),
                        np.asarray(g_inst_o).ravel() * INST_UNITS])
    scale = float(np.max(np.abs(b)))
    if scale == 0.0:
        assert float(np.max(np.abs(a))) == 0.0, what
        return 0.0
    err = float(np.max(np.abs(a - b))) / scale
    assert err <= tol, f"{what}: ||diff||/||g|| = {err:.3e}"
    big = np.abs(b) >= 1e-3 * scale
    rel = np.abs(a[big] - b[big]) / np.abs(b[big])
    worst = float(np.max(rel)) if rel.size else 0.0
    assert worst <= tol, f"{what}: component rel err {worst:.3e}"
    return max(err, worst)
