"""Pins of the CPU oracle against facts other than itself.

Each test checks the oracle against a closed form, an invariant of the
physics, an independent re-derivation (other recursion, other frame, other
formulation, higher precision) or a library routine for a special case.  The
forward model is the Abeles formalism named in Sec. 2.1 of the paper, with the
conventions stated in the oracle's header.
"""
import math

import mpmath
import numpy as np
import pytest

FOURPI = 4.0 * math.pi


def rand_stack(rng, L, sigma=True, absorb=True, rho_lo=-0.5e-6, rho_hi=6.5e-6,
               d_lo=10.0, d_hi=300.0, backing=2.07e-6, fronting=0.0):
    rows = np.zeros((L + 2, 4))
    rows[0, 1] = fronting
    rows[1:L + 1, 0] = rng.uniform(d_lo, d_hi, L)
    rows[1:L + 1, 1] = rng.uniform(rho_lo, rho_hi, L)
    if absorb:
        rows[1:L + 1, 2] = rng.uniform(0.0, 1e-8, L)
    rows[L + 1, 1] = backing
    if sigma:
        rows[1:, 3] = rng.uniform(1.0, 15.0, L + 1)
    return rows


def rel(a, b):
    a = np.asarray(a, dtype=float)
    b = np.asarray(b, dtype=float)
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))


# ---------------------------------------------------------------- kz root ----

def test_kz_root_branch_matches_mpmath(orc):
    """Root with Re >= 0, Im <= 0 (signed-zero cut) vs mpmath at 50 digits."""
    rng = np.random.default_rng(1)
    mpmath.mp.dps = 50
    for _ in range(200):
        x = rng.uniform(-1e-4, 1e-4)
        y = -abs(rng.uniform(0, 1e-6)) * rng.integers(0, 2)
        if y == 0.0:
            y = -0.0
        k = orc.kz(x, y)
        # physical root of conj(w) is principal; ours is its conjugate
        kp = mpmath.sqrt(mpmath.mpc(x, -y if y != 0 else 0.0))
        ref = complex(kp.real, -kp.imag)
        assert k.real >= 0.0 and math.copysign(1.0, k.imag) <= 0 or k.imag == 0.0
        assert abs(k - ref) <= 4.5e-16 * abs(ref) + 1e-300
    # on the cut: w real negative with no absorption -> -i sqrt|w|
    k = orc.kz(-4e-6, -0.0)
    assert k.real == 0.0 and k.imag == pytest.approx(-2e-3, rel=1e-15)


# ------------------------------------------------------- Fresnel / NC -------

def _fresnel_nc_mp(q, rho0, rho1, rho1_im, sigma):
    """Single interface: R = |(k0-k1)/(k0+k1)|^2 exp(-4 Re(k0 k1) sigma^2),
    physical frame, at the caller's mpmath precision."""
    q = mpmath.mpf(q)
    k0 = q / 2
    w1 = k0 ** 2 - 4 * mpmath.pi * (mpmath.mpf(rho1) - mpmath.mpf(rho0)) \
        + 1j * 4 * mpmath.pi * abs(mpmath.mpf(rho1_im))
    k1 = mpmath.sqrt(w1)
    r = (k0 - k1) / (k0 + k1)
    return abs(r) ** 2 * mpmath.exp(-4 * mpmath.re(k0 * k1) * mpmath.mpf(sigma) ** 2)


@pytest.mark.parametrize("rho1,rho1_im,sigma", [
    (2.07e-6, 0.0, 0.0), (2.07e-6, 0.0, 5.0), (6.35e-6, 3e-7, 8.0),
    (-0.56e-6, 0.0, 3.0), (4.0e-6, 1e-8, 12.0)])
def test_single_interface_closed_form(orc, rho1, rho1_im, sigma):
    q = np.geomspace(0.002, 0.4, 157)
    rows = np.array([[0, 0.0, 0, 0], [0, rho1, rho1_im, sigma]], float)
    R = orc.reflectivity(rows, q)
    mpmath.mp.dps = 50
    ref = np.array([float(_fresnel_nc_mp(qi, 0.0, rho1, rho1_im, sigma)) for qi in q])
    # The plain definition forms kz0 - kz1, which cancels at high Q: its
    # relative rounding error is about eps * |kz0| / |kz0 - kz1| (<= 3e3 eps
    # on this grid), so the bound is 2e-11, not eps.
    assert rel(R, ref) < 2e-11


def test_nonzero_fronting_sld_closed_form(orc):
    q = np.geomspace(0.004, 0.3, 61)
    rows = np.array([[0, 1.1e-6, 5e-7, 0], [0, 4.5e-6, 2e-8, 6.0]], float)
    R = orc.reflectivity(rows, q)
    mpmath.mp.dps = 50
    ref = np.array([float(_fresnel_nc_mp(qi, 1.1e-6, 4.5e-6, 2e-8, 6.0)) for qi in q])
    # the fronting rho_im is ignored by the model
    assert rel(R, ref) < 2e-11


# ------------------------------------------------- total reflection ---------

def test_total_reflection_below_backing_edge(orc):
    """R = 1 below the backing's critical edge for real SLDs, any N, any NC."""
    rng = np.random.default_rng(2)
    for L in [0, 1, 2, 5, 12, 30]:
        rows = rand_stack(rng, L, sigma=True, absorb=False, backing=6.35e-6)
        qc = 2.0 * math.sqrt(FOURPI * (rows[-1, 1] - rows[0, 1]))
        q = np.linspace(0.02 * qc, 0.999 * qc, 60)
        R = orc.reflectivity(rows, q)
        assert np.max(np.abs(R - 1.0)) < 5e-13, L


def test_passive_stack_R_at_most_one(orc):
    rng = np.random.default_rng(3)
    q = np.geomspace(0.003, 0.4, 300)
    for L in [1, 4, 10]:
        rows = rand_stack(rng, L, sigma=False, absorb=True)
        R = orc.reflectivity(rows, q)
        assert np.all(R <= 1.0 + 1e-13)


# ------------------------------------------------- thick absorber -----------

def test_thick_absorber_selects_decaying_branch(orc):
    """Below a strongly absorbing, very thick layer nothing returns: R equals
    the top interface's NC-Fresnel value.  A root on the wrong branch would
    make the buried term grow instead of decay."""
    q = np.geomspace(0.02, 0.3, 50)
    rim, d = 5e-5, 2e4
    top = np.array([[0, 0.0, 0, 0], [0, 3.0e-6, rim, 4.0]], float)
    stack = np.array([[0, 0.0, 0, 0], [d, 3.0e-6, rim, 4.0],
                      [0, 6.0e-6, 0.0, 9.0]], float)
    # the buried path is negligible: |exp(-2 i kz d)| < 1e-30 on the grid
    for qi in q:
        k = orc.kz(0.25 * qi * qi - FOURPI * 3.0e-6, -FOURPI * rim)
        assert math.exp(2.0 * k.imag * d) < 1e-30
    assert rel(orc.reflectivity(stack, q), orc.reflectivity(top, q)) < 1e-13


# ------------------------------------------ independent re-derivations ------

@pytest.mark.parametrize("L", [0, 1, 2, 5, 10, 20, 40])
def test_abeles_equals_parratt(orc, L):
    """Abeles product (Im kz <= 0 frame) vs Parratt recursion written in the
    physical frame with library principal roots."""
    rng = np.random.default_rng(100 + L)
    q = np.geomspace(0.003, 0.4, 200)
    for _ in range(3):
        rows = rand_stack(rng, L)
        assert rel(orc.reflectivity(rows, q), orc.reflectivity_parratt(rows, q)) < 1e-12


@pytest.mark.parametrize("L", [0, 1, 3, 8])
def test_abeles_equals_boundary_matching_solve(orc, L):
    """sigma = 0: R from the 2(N+1) continuity equations solved by LU."""
    rng = np.random.default_rng(200 + L)
    q = np.geomspace(0.004, 0.35, 120)
    for _ in range(3):
        rows = rand_stack(rng, L, sigma=False)
        assert rel(orc.reflectivity(rows, q), orc.reflectivity_linsys(rows, q)) < 1e-10


def _parratt_mp(rows, q):
    mpmath.mp.dps = 50
    N = rows.shape[0] - 2
    q = mpmath.mpf(q)
    k = [q / 2]
    rho0 = mpmath.mpf(rows[0, 1])
    for j in range(1, N + 2):
        w = q * q / 4 - 4 * mpmath.pi * (mpmath.mpf(rows[j, 1]) - rho0) \
            + 1j * 4 * mpmath.pi * abs(mpmath.mpf(rows[j, 2]))
        k.append(mpmath.sqrt(w))

    def rr(j):
        rf = (k[j] - k[j + 1]) / (k[j] + k[j + 1]) if k[j] != k[j + 1] else mpmath.mpc(0)
        return rf * mpmath.exp(-2 * k[j] * k[j + 1] * mpmath.mpf(rows[j + 1, 3]) ** 2)

    X = rr(N)
    for j in range(N - 1, -1, -1):
        Y = X * mpmath.exp(2j * k[j + 1] * mpmath.mpf(rows[j + 1, 0]))
        X = (rr(j) + Y) / (1 + rr(j) * Y)
    return abs(X) ** 2


def test_fifty_digit_reference(orc):
    rng = np.random.default_rng(4)
    q = np.geomspace(0.005, 0.3, 25)
    for L in [1, 2, 3]:
        rows = rand_stack(rng, L)
        ref = np.array([float(_parratt_mp(rows, qi)) for qi in q])
        assert rel(orc.reflectivity(rows, q), ref) < 5e-13


def test_high_precision_reference_module(orc):
    """oracle/mp_reference.py (the 50-digit reference used for the deep-stack
    fixtures): at one interface it is the Fresnel / Nevot-Croce closed form
    at the same precision; on shallow stacks the FP64 Abeles oracle agrees
    with it to rounding."""
    from oracle import mp_reference
    mpmath.mp.dps = 50
    for rho1, im1, sig in [(2.07e-6, 0.0, 5.0), (6.35e-6, 3e-7, 8.0), (-0.56e-6, 0.0, 3.0)]:
        rows = np.array([[0, 0.0, 0, 0], [0, rho1, im1, sig]], float)
        for qi in (0.004, 0.011, 0.05, 0.2):
            a = mp_reference.parratt_R(rows, qi)
            b = _fresnel_nc_mp(qi, 0.0, rho1, im1, sig)
            assert abs(a - b) <= mpmath.mpf("1e-40") * abs(b)
    rng = np.random.default_rng(5)
    q = np.geomspace(0.005, 0.3, 9)
    for L in [1, 4, 12]:
        rows = rand_stack(rng, L)
        ref = np.array([float(mp_reference.parratt_R(rows, qi)) for qi in q])
        assert rel(orc.reflectivity(rows, q), ref) < 5e-12


# ------------------------------------------------------------ invariances ---

def test_split_layer_invariance(orc):
    rng = np.random.default_rng(5)
    q = np.geomspace(0.004, 0.35, 150)
    for L in [1, 3, 7]:
        rows = rand_stack(rng, L)
        j = int(rng.integers(1, L + 1))
        half = rows[j].copy()
        half[0] *= 0.5
        other = half.copy()
        other[3] = 37.0  # roughness between identical halves must not matter
        split = np.vstack([rows[:j], half[None], other[None], rows[j + 1:]])
        assert rel(orc.reflectivity(split, q), orc.reflectivity(rows, q)) < 1e-12


def test_zero_thickness_insert_copying_a_neighbour(orc):
    rng = np.random.default_rng(6)
    q = np.geomspace(0.004, 0.35, 150)
    rows = rand_stack(rng, 4)
    R0 = orc.reflectivity(rows, q)
    j = 2  # insert between medium 1 and 2
    # (a) copy of the medium above; its own interface roughness arbitrary
    ins = rows[j - 1].copy()
    ins[0] = 0.0
    ins[3] = 23.0
    s = np.vstack([rows[:j], ins[None], rows[j:]])
    assert rel(orc.reflectivity(s, q), R0) < 1e-12
    # (b) copy of the medium below: takes over the interface roughness, and
    #     the roughness between it and its twin is arbitrary
    ins = rows[j].copy()
    ins[0] = 0.0
    ins[3] = rows[j, 3]
    below = rows[j].copy()
    below[3] = 17.0
    s = np.vstack([rows[:j], ins[None], below[None], rows[j + 1:]])
    assert rel(orc.reflectivity(s, q), R0) < 1e-12


def test_zero_thickness_insert_without_roughness(orc):
    """Any SLD at zero thickness is invisible when every sigma is 0
    (addition theorem of the Fresnel coefficients)."""
    rng = np.random.default_rng(7)
    q = np.geomspace(0.004, 0.35, 150)
    rows = rand_stack(rng, 3, sigma=False)
    ins = np.array([0.0, 9.9e-6, 3e-7, 0.0])
    s = np.vstack([rows[:2], ins[None], rows[2:]])
    assert rel(orc.reflectivity(s, q), orc.reflectivity(rows, q)) < 1e-11


def test_thickness_periodicity(orc):
    """A layer with real kz_j: R(d_j + pi/kz_j) = R(d_j) at fixed Q."""
    rng = np.random.default_rng(8)
    rows = rand_stack(rng, 5)
    j = 3
    rows[j, 2] = 0.0
    rows[j, 1] = 1.0e-6
    for qv in [0.03, 0.08, 0.2, 0.33]:
        k = orc.kz(0.25 * qv * qv - FOURPI * (rows[j, 1] - rows[0, 1]), -0.0)
        assert k.imag == 0.0 and k.real > 0
        shifted = rows.copy()
        shifted[j, 0] += math.pi / k.real
        a = orc.reflectivity(rows, [qv])[0]
        b = orc.reflectivity(shifted, [qv])[0]
        assert abs(a - b) <= 1e-11 * a


def test_kiessig_fringe_period(orc):
    """Single film on a substrate, sigma = 0: fringes are periodic in
    Q1 = 2 kz_1 with period 2 pi / d."""
    d = 800.0
    rows = np.array([[0, 0.0, 0, 0], [d, 4.0e-6, 0, 0], [0, 2.07e-6, 0, 0]], float)
    q = np.linspace(0.15, 0.30, 200001)
    R = orc.reflectivity(rows, q)
    q1 = 2.0 * np.sqrt(0.25 * q * q - FOURPI * 4.0e-6)
    mins = np.where((R[1:-1] < R[:-2]) & (R[1:-1] < R[2:]))[0] + 1
    spacing = np.diff(q1[mins])
    assert len(spacing) > 10
    assert np.max(np.abs(spacing - 2 * math.pi / d)) < 0.01 * 2 * math.pi / d


def test_reciprocity(orc):
    """Lossless stack, sigma = 0: reflectance seen from either side is equal,
    with the momentum transfer measured in the incidence medium."""
    rng = np.random.default_rng(9)
    rows = rand_stack(rng, 6, sigma=False, absorb=False, rho_lo=0.5e-6, rho_hi=4e-6)
    rows[0, 1] = 0.0
    rows[-1, 1] = 2.07e-6
    rev = rows[::-1].copy()
    q = np.geomspace(0.03, 0.3, 80)
    kN = np.sqrt(0.25 * q * q - FOURPI * (rows[-1, 1] - rows[0, 1]))
    Rf = orc.reflectivity(rows, q)
    Rb = orc.reflectivity(rev, 2.0 * kN)
    assert rel(Rb, Rf) < 1e-11


# ------------------------------------------------------------- smearing -----

def test_gauss_legendre_nodes_against_library_and_exactness(orc):
    x, u = orc.gauss_legendre17()
    xn, un = np.polynomial.legendre.leggauss(17)
    assert np.max(np.abs(x - xn)) < 4e-16
    assert np.max(np.abs(u - un)) < 4e-15
    for m in range(0, 34):
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        assert abs(np.dot(u, x ** m) - exact) < 2e-15
    assert x[8] == 0.0
    assert np.array_equal(x[:8], -x[:8:-1]) and np.array_equal(u[:8], u[:8:-1])


def test_smear_rule_moments(orc):
    t, w = orc.smear_rule(0.05)
    assert len(t) == 17
    assert abs(w.sum() - 1.0) < 2e-16 * 17
    assert abs(np.dot(w, t)) < 1e-16
    # discrete rule vs the continuous Gaussian truncated at +-3.5 sigma
    a = 3.5
    phi = math.exp(-a * a / 2) / math.sqrt(2 * math.pi)
    Phi = 0.5 * (1 + math.erf(a / math.sqrt(2)))
    var_trunc = 1.0 - 2 * a * phi / (2 * Phi - 1)
    assert abs(np.dot(w, t * t) - var_trunc) < 1e-9
    t0, w0 = orc.smear_rule(0.0)
    assert list(t0) == [0.0] and list(w0) == [1.0]


def test_smear_nodes_width(orc):
    Q = np.array([0.01, 0.1, 0.3])
    nodes = orc.smear_nodes(Q, 0.08)
    t, w = orc.smear_rule(0.08)
    sig = 0.08 * Q / (2 * math.sqrt(2 * math.log(2)))
    assert np.allclose((nodes - Q[:, None]) / sig[:, None], t[None, :], rtol=1e-13, atol=1e-13)
    assert np.all(nodes[:, 8] == Q)


def test_smearing_keeps_total_reflection(orc):
    """Where every node lies below the edge, R = 1 for each, so R_sm = 1."""
    rng = np.random.default_rng(10)
    rows = rand_stack(rng, 4, absorb=False, backing=6.35e-6)
    qc = 2.0 * math.sqrt(FOURPI * 6.35e-6)
    Q = np.linspace(0.2 * qc, 0.8 * qc, 20)
    assert np.max(np.abs(orc.smeared(rows, Q, 0.05) - 1.0)) < 1e-13


def test_smearing_small_width_limit(orc):
    rng = np.random.default_rng(11)
    rows = rand_stack(rng, 3)
    Q = np.geomspace(0.02, 0.3, 30)
    R = orc.reflectivity(rows, Q)
    for dqq in [1e-3, 1e-4]:
        Rs = orc.smeared(rows, Q, dqq)
        assert rel(Rs, R) < 5e3 * dqq ** 2 + 1e-12
    assert np.array_equal(orc.smeared(rows, Q, 0.0), R)


def test_smearing_is_the_weighted_node_average(orc):
    rng = np.random.default_rng(12)
    rows = rand_stack(rng, 5)
    Q = np.geomspace(0.006, 0.3, 25)
    t, w = orc.smear_rule(0.05)
    nodes = orc.smear_nodes(Q, 0.05)
    Rn = orc.reflectivity(rows, nodes.reshape(-1)).reshape(nodes.shape)
    assert rel(orc.smeared(rows, Q, 0.05), Rn @ w) < 1e-14


# ------------------------------------------------------ instrument / logL ---

def _data(orc, rows, Q, dqq, scale=1.0, bkg=1e-7, seed=13, off=1.03):
    Rm = orc.model_curve(rows, scale, bkg, Q, dqq)
    rng = np.random.default_rng(seed)
    e = 0.03 * Rm
    Robs = off * Rm + e * rng.standard_normal(Q.size)
    return Robs, e


def test_instrument_scale_and_background(orc):
    rng = np.random.default_rng(14)
    rows = rand_stack(rng, 4)
    Q = np.geomspace(0.005, 0.35, 40)
    Rs = orc.smeared(rows, Q, 0.05)
    assert rel(orc.model_curve(rows, 1.3, 2e-6, Q, 0.05), 1.3 * Rs + 2e-6) < 1e-15


def test_loglik_perfect_fit_and_chi2(orc):
    rng = np.random.default_rng(15)
    rows = rand_stack(rng, 4)
    Q = np.geomspace(0.005, 0.35, 40)
    Rm = orc.model_curve(rows, 0.97, 3e-7, Q, 0.05)
    e = 0.03 * Rm + 1e-9
    ll = orc.loglik(rows, 0.97, 3e-7, Q, Rm, e, 0.05)
    const = -np.sum(np.log(e)) - 0.5 * Q.size * math.log(2 * math.pi)
    assert abs(ll - const) <= 1e-13 * abs(const)
    Robs, e = _data(orc, rows, Q, 0.05)
    chi2 = np.sum((orc.model_curve(rows, 1.0, 1e-7, Q, 0.05) - Robs) ** 2 / e ** 2)
    ll = orc.loglik(rows, 1.0, 1e-7, Q, Robs, e, 0.05)
    const = -np.sum(np.log(e)) - 0.5 * Q.size * math.log(2 * math.pi)
    assert abs(ll - (-0.5 * chi2 + const)) <= 1e-12 * abs(ll)


def test_instrument_gradient_closed_form(orc):
    rng = np.random.default_rng(16)
    rows = rand_stack(rng, 6)
    Q = np.geomspace(0.005, 0.35, 50)
    Robs, e = _data(orc, rows, Q, 0.05)
    scale, bkg = 1.04, 2e-7
    _, _, gi = orc.loglik_grad_cs(rows, scale, bkg, Q, Robs, e, 0.05)
    Rsm = orc.smeared(rows, Q, 0.05)
    ghat = -(scale * Rsm + bkg - Robs) / e ** 2
    assert abs(gi[1] - ghat.sum()) <= 1e-12 * np.abs(ghat).sum()
    assert abs(gi[0] - np.dot(ghat, Rsm)) <= 1e-12 * np.abs(ghat * Rsm).sum()


# ------------------------------------------------------------- gradient -----

def _scaled_err(g, gref):
    """Gradient error in natural units (d, sigma: 1 A; rho: 1e-6 A^-2)."""
    s = np.array([1.0, 1e-6, 1e-6, 1.0])
    a = g * s
    b = gref * s
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


@pytest.mark.parametrize("L,dqq", [(1, 0.0), (3, 0.05), (6, 0.03)])
def test_complex_step_matches_richardson(orc, L, dqq):
    rng = np.random.default_rng(300 + L)
    rows = rand_stack(rng, L)
    rows[1:, 2] = rng.uniform(2e-8, 5e-8, L + 1)  # keep FD steps off the |x| kink
    Q = np.geomspace(0.006, 0.3, 30)
    Robs, e = _data(orc, rows, Q, dqq)
    ll, g, gi = orc.loglik_grad_cs(rows, 1.02, 1.5e-7, Q, Robs, e, dqq)
    gf, gif = orc.loglik_grad_fd(rows, 1.02, 1.5e-7, Q, Robs, e, dqq, rel_step=1e-4)
    assert _scaled_err(g, gf) < 1e-7
    assert rel(gi, gif) < 1e-7
    # entries the model does not read
    assert g[0, 0] == 0 and g[0, 2] == 0 and g[0, 3] == 0 and g[-1, 0] == 0


def test_single_interface_derivatives_closed_form(orc):
    """dR/dsigma = -8 Re(kz0 kz1) sigma R; dR/drho1 from the 50-digit closed
    form by numerical differentiation in mpmath."""
    q = np.geomspace(0.012, 0.3, 12)
    rho1, sig = 3.0e-6, 6.0
    rows = np.array([[0, 0.0, 0, 0], [0, rho1, 0.0, sig]], float)
    J = orc.reflectivity_jac_cs(rows, q)
    R = orc.reflectivity(rows, q)
    for i, qi in enumerate(q):
        k0 = 0.5 * qi
        k1 = orc.kz(0.25 * qi * qi - FOURPI * rho1, -0.0)
        ref_sig = -8.0 * (k0 * k1).real * sig * R[i]
        assert abs(J[i, 1, 3] - ref_sig) <= 1e-12 * abs(ref_sig) + 1e-18
    mpmath.mp.dps = 50
    dref = np.array([float(mpmath.diff(lambda x: _fresnel_nc_mp(qi, 0.0, x, 0.0, sig),
                                       mpmath.mpf(rho1))) for qi in q])
    # below the edge R == 1 and the derivative is 0: compare on the scale of
    # the largest derivative on the grid
    assert np.max(np.abs(J[:, 1, 1] - dref)) <= 1e-11 * np.max(np.abs(dref))


def test_translation_invariance_of_sld_gradient(orc):
    """Shifting every real SLD (fronting included) by the same amount leaves
    R unchanged, so the rho_re gradient sums to zero over all rows."""
    rng = np.random.default_rng(17)
    for L in [0, 2, 9]:
        rows = rand_stack(rng, L)
        Q = np.geomspace(0.006, 0.3, 20)
        Robs, e = _data(orc, rows, Q, 0.05)
        _, g, _ = orc.loglik_grad_cs(rows, 1.0, 1e-7, Q, Robs, e, 0.05)
        assert abs(g[:, 1].sum()) <= 1e-12 * np.abs(g[:, 1]).max()


def test_split_layer_gradient_identities(orc):
    rng = np.random.default_rng(18)
    rows = rand_stack(rng, 4)
    j = 2
    half = rows[j].copy()
    half[0] *= 0.5
    other = half.copy()
    other[3] = 11.0
    split = np.vstack([rows[:j], half[None], other[None], rows[j + 1:]])
    Q = np.geomspace(0.006, 0.3, 25)
    Robs, e = _data(orc, rows, Q, 0.05)
    _, g, gi = orc.loglik_grad_cs(rows, 1.0, 1e-7, Q, Robs, e, 0.05)
    _, gs, gis = orc.loglik_grad_cs(split, 1.0, 1e-7, Q, Robs, e, 0.05)
    tol = 1e-10
    assert abs(gs[j, 0] - g[j, 0]) <= tol * abs(g[j, 0])
    assert abs(gs[j + 1, 0] - g[j, 0]) <= tol * abs(g[j, 0])
    assert abs(gs[j, 1] + gs[j + 1, 1] - g[j, 1]) <= tol * abs(g[j, 1])
    assert abs(gs[j, 2] + gs[j + 1, 2] - g[j, 2]) <= tol * abs(g[j, 2])
    assert gs[j + 1, 3] == 0.0
    assert abs(gs[j, 3] - g[j, 3]) <= tol * abs(g[j, 3])
    assert rel(gis, gi) < 1e-12


def test_gradient_periodic_in_thickness(orc):
    rng = np.random.default_rng(19)
    rows = rand_stack(rng, 4)
    j = 2
    rows[j, 2] = 0.0
    rows[j, 1] = 1.5e-6
    qv = 0.12
    k = orc.kz(0.25 * qv * qv - FOURPI * rows[j, 1], -0.0)
    shifted = rows.copy()
    shifted[j, 0] += math.pi / k.real
    a = orc.reflectivity_jac_cs(rows, [qv])[0]
    b = orc.reflectivity_jac_cs(shifted, [qv])[0]
    mask = np.ones_like(a, bool)
    mask[j, 1] = False   # dR/drho_j picks up d_j * dkz/drho from the phase
    mask[j, 2] = False
    mask[0, 1] = False   # equals minus the sum of the others, includes rho_j
    scale = np.max(np.abs(a[mask] * np.where(np.arange(4) % 3 == 0, 1.0, 1e-6)[None, :].repeat(a.shape[0], 0)[mask]))
    diff = np.abs(a - b) * np.where(np.arange(4) % 3 == 0, 1.0, 1e-6)[None, :]
    assert np.max(diff[mask]) <= 1e-9 * scale
