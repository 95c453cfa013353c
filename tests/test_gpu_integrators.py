"""GPU parity of the rows around the gradient: HMC leapfrog (eager and
captured in a HIP graph), the VI reparameterised ELBO gradient and the co-fit
tie-sum, against the oracle (oracle/integrators.py driven by oracle
gradients) through the C ABI."""
import numpy as np
import pytest

from nr_check import G_TOL

pytestmark = pytest.mark.gpu

UNITS = np.array([1.0, 1e-6, 1e-6, 1.0])  # natural units of d, rho_re, rho_im, sigma


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def nr(torch_cuda):
    import paper_2509_06924_amd as nr
    return nr


def _batch(seed, n_items=3, L_choices=(1, 3, 4), nq=(45, 70)):
    from paper_2509_06924_amd import inputs
    rng = np.random.default_rng(seed)
    return inputs.random_batch(rng, n_items=n_items, L_choices=list(L_choices),
                               nq_choices=list(nq), dqq_choices=[0.05], n_datasets=2)


def _flat(batch, rows, scale, bkg):
    """theta vector of every item: rows (packed) then the instrument pairs."""
    return np.concatenate([rows.reshape(-1), np.stack([scale, bkg], 1).reshape(-1)])


def _oracle_grad_fn(orc, batch):
    nre = batch.layers.size

    def grad(theta):
        rows = theta[:nre].reshape(-1, 4)
        inst = theta[nre:].reshape(-1, 2)
        g = np.zeros_like(theta)
        gr = g[:nre].reshape(-1, 4)
        gi = g[nre:].reshape(-1, 2)
        for b in range(batch.n_items):
            r0, r1 = batch.row_off[b], batch.row_off[b + 1]
            Q, Robs, Rerr, dqq = batch.data_of(b)
            _, gg, ggi = orc.loglik_grad_cs(rows[r0:r1], inst[b, 0], inst[b, 1], Q, Robs, Rerr, dqq)
            gr[r0:r1] = gg
            gi[b] = ggi
        return g
    return grad


def _masses(batch):
    im_rows = np.tile(UNITS ** 2, (batch.layers.shape[0], 1))
    im_inst = np.tile(np.array([1.0, 1e-14]), (batch.n_items, 1))
    return im_rows, im_inst


def _moving_mask(batch):
    """Entries the model reads (the drift moves only these)."""
    m = np.zeros_like(batch.layers, bool)
    for b in range(batch.n_items):
        r0, r1 = batch.row_off[b], batch.row_off[b + 1]
        m[r0, 1] = True
        m[r0 + 1:r1 - 1, :] = True
        m[r1 - 1, 1:] = True
    return m


def _state(nr, batch, seed):
    prob = nr.Problem.from_batch(batch)
    rng = np.random.default_rng(seed)
    mom_rows = rng.standard_normal(batch.layers.shape) / UNITS
    mom_inst = rng.standard_normal((batch.n_items, 2)) / np.array([1.0, 1e-7])
    im_rows, im_inst = _masses(batch)
    st = nr.HmcState(prob, mom_rows, mom_inst, im_rows, im_inst)
    return prob, st, mom_rows, mom_inst, im_rows, im_inst


def _cmp(a, b, scale, tol, what):
    err = np.max(np.abs(a - b) / scale)
    assert err <= tol, f"{what}: {err:.3e}"


@pytest.mark.parametrize("n_steps", [1, 3])
def test_leapfrog_matches_oracle(nr, orc, torch_cuda, n_steps):
    from oracle import integrators as oi
    batch = _batch(21)
    prob, st, mom_rows, mom_inst, im_rows, im_inst = _state(nr, batch, 5)
    dt = 2e-3
    prob.leapfrog(st, dt, n_steps)
    torch_cuda.cuda.synchronize()
    theta0 = _flat(batch, batch.layers, batch.scale, batch.bkg)
    r0 = np.concatenate([mom_rows.reshape(-1), mom_inst.reshape(-1)])
    mask = np.concatenate([_moving_mask(batch).reshape(-1), np.ones(2 * batch.n_items, bool)])
    im = np.concatenate([im_rows.reshape(-1), im_inst.reshape(-1)]) * mask
    th, r, _ = oi.leapfrog(theta0, r0, _oracle_grad_fn(orc, batch), dt, n_steps, inv_mass=im)
    th_k = _flat(batch, st.layers.cpu().numpy(), st.scale.cpu().numpy(), st.bkg.cpu().numpy())
    r_k = np.concatenate([st.mom_rows.cpu().numpy().reshape(-1), st.mom_inst.cpu().numpy().reshape(-1)])
    units = np.concatenate([np.tile(UNITS, batch.layers.shape[0]),
                            np.tile([1.0, 1e-7], batch.n_items)])
    # positions: the displacement is dt M^-1 times the summed momenta, which
    # carry the gradient; to first order its error is the gradient tolerance
    # times the displacement (plus rounding of the position itself)
    disp = np.max(np.abs((th - theta0) / units))
    _cmp(th_k, th, units, G_TOL * disp + 1e-12, "positions")
    # momenta in units of 1/natural unit, relative to the largest
    rs = np.max(np.abs(r * units))
    _cmp(r_k * units, r * units, rs, G_TOL, "momenta")
    # frozen / unread entries did not move
    assert np.array_equal(th_k[~mask], theta0[~mask])


def _nearfit_batch(orc, seed, Ls=(1, 3, 4), nq=60):
    """Items evaluated within 1 % of the truth draw their data came from."""
    from paper_2509_06924_amd import inputs
    rng = np.random.default_rng(seed)
    ds, its = [], []
    for b, L in enumerate(Ls):
        truth = inputs.draw_stack(rng, L)
        # logL depends on |rho_im|, whose gradient jumps at rho_im = 0: a
        # rounding-level difference of a retraced position would pick the
        # other one-sided gradient, so every medium starts off the kink
        truth[1:, 2] = np.maximum(truth[1:, 2], 5e-9)
        Q = inputs.log_grid(0.005, 0.35, nq)
        R = orc.model_curve(truth, 1.0, 1e-7, Q, 0.05)
        e = 0.03 * R
        ds.append((Q, R + e * rng.standard_normal(nq), e, 0.05))
        near = truth * (1 + 0.01 * rng.uniform(-1, 1, truth.shape))
        near[0, [0, 2, 3]] = 0.0
        near[-1, 0] = 0.0
        its.append((b, near, 1.0, 1e-7))
    return inputs._pack("nearfit", ds, its, {})


@pytest.mark.parametrize("data", ["synthetic", "nearfit"])
def test_leapfrog_reversible(nr, orc, torch_cuda, data):
    """Ten steps forward, momenta negated, ten steps back: every position and
    momentum returns to 1e-12 relative (measured: 2e-13 / 6e-13 on the
    synthetic data, 1e-15 / 7e-15 near the fit)."""
    if data == "synthetic":
        batch = _batch(22)
        # the backings are drawn with rho_im = 0 exactly (see _nearfit_batch)
        batch.layers[batch.row_off[1:] - 1, 2] = 5e-9
    else:
        batch = _nearfit_batch(orc, 5)
    prob, st, *_ = _state(nr, batch, 6)
    x0 = st.layers.clone()
    r0 = st.mom_rows.clone()
    prob.leapfrog(st, 1e-3, 10)
    st.mom_rows.neg_()
    st.mom_inst.neg_()
    prob.leapfrog(st, 1e-3, 10)
    torch_cuda.cuda.synchronize()
    units = torch_cuda.tensor(UNITS, dtype=torch_cuda.float64, device="cuda")
    moved = x0 != 0
    rel = ((st.layers - x0).abs() / x0.abs().clamp_min(1e-300))[moved]
    assert float(rel.max()) < 1e-12
    rs = float((r0 * units).abs().max())
    assert float(((st.mom_rows + r0) * units).abs().max()) < 1e-12 * rs


def test_leapfrog_graph_replays_equal_eager(nr, torch_cuda):
    torch = torch_cuda
    batch = _batch(23)
    prob_e, st_e, *_ = _state(nr, batch, 7)
    prob_g, st_g, *_ = _state(nr, batch, 7)
    graph = nr.LeapfrogGraph(prob_g, st_g, 1e-3, 4)
    for rep in range(3):
        prob_e.leapfrog(st_e, 1e-3, 4)
        graph.launch()
        torch.cuda.synchronize()
        for a, b in [(st_e.layers, st_g.layers), (st_e.mom_rows, st_g.mom_rows),
                     (st_e.mom_inst, st_g.mom_inst), (st_e.g_rows, st_g.g_rows),
                     (st_e.logL, st_g.logL), (st_e.scale, st_g.scale)]:
            assert torch.equal(a, b), f"replay {rep} differs from eager"
        # the program's own eager work between replays
        _ = (st_e.layers * 2.0).sum().item()
    graph.close()


def test_vi_elbo_gradient_matches_oracle(nr, orc, torch_cuda):
    from oracle import integrators as oi
    from paper_2509_06924_amd import inputs
    rng = np.random.default_rng(31)
    L, S = 3, 6
    mu_rows = inputs.draw_stack(rng, L)
    Q = inputs.log_grid(0.005, 0.35, 60)
    Robs, err = inputs.synthetic_curve(Q, rng)
    P = (L + 2) * 4 + 2
    mu = np.concatenate([mu_rows.reshape(-1), [1.0, 1e-7]])
    omega = np.full(P, -3.0)
    mask = np.zeros(P, np.uint8)
    mask[4:4 * (L + 1)] = 1   # finite layers
    mask[-2:] = 1              # scale, bkg
    scal = np.concatenate([np.tile(UNITS, L + 2), [1.0, 1e-7]])
    eps = rng.standard_normal((S, P))
    # per-entry scale of the noise: omega such that s = 1e-3 natural unit
    omega = np.log(np.expm1(1e-3 * scal))
    batch = inputs._pack("vi", [(Q, Robs, err, 0.05)],
                         [(0, mu_rows.copy(), 1.0, 1e-7) for _ in range(S)], {})
    prob = nr.Problem.from_batch(batch)
    elbo, gmu, gom, ll = prob.vi_elbo_grad(mu, omega, mask, eps)
    torch_cuda.cuda.synchronize()

    def f(th):
        rows = th[:-2].reshape(-1, 4)
        l, g, gi = orc.loglik_grad_cs(rows, th[-2], th[-1], Q, Robs, err, 0.05)
        return l, np.concatenate([g.reshape(-1), gi])

    elbo_o, gmu_o, gom_o, ll_o = oi.vi_elbo_grad(mu, omega, mask, eps, f)
    assert abs(float(elbo.cpu()[0]) - elbo_o) <= 1e-9 * abs(elbo_o)
    assert np.allclose(ll.cpu().numpy(), ll_o, rtol=1e-9, atol=0)
    gm = gmu.cpu().numpy()
    assert np.max(np.abs((gm - gmu_o) * scal)) <= G_TOL * np.max(np.abs(gmu_o * scal))
    go = gom.cpu().numpy()
    assert np.max(np.abs(go - gom_o)) <= G_TOL * np.max(np.abs(gom_o))
    assert np.all(gm[mask == 0] == 0) and np.all(go[mask == 0] == 0)


def test_tie_sum_cofit(nr, torch_cuda):
    torch = torch_cuda
    from paper_2509_06924_amd import inputs
    batch = inputs.c3_cofit(n_draws=4, nqs=(25, 30, 35), L=3)
    prob = nr.Problem.from_batch(batch)
    _, g_rows, g_inst = prob.loglik_grad()
    # shared parameters per draw: every row entry except the backing rho_re
    # (the contrast), plus the background; scale is fixed
    rows = batch.row_off[1] - batch.row_off[0]
    per_draw = rows * 4 - 1 + 1
    n_out = 4 * per_draw
    nre = batch.layers.size
    tie = -np.ones(nre + 2 * batch.n_items, np.int64)
    for b in range(batch.n_items):
        d = b // 3
        k = 0
        for r in range(rows):
            for f in range(4):
                if r == rows - 1 and f == 1:
                    continue
                tie[(batch.row_off[b] + r) * 4 + f] = d * per_draw + k
                k += 1
        tie[nre + 2 * b + 1] = d * per_draw + k
    first, src = nr.tie_map_to_csr(tie, n_out)
    vals = torch.cat([g_rows.reshape(-1), g_inst.reshape(-1)])
    out = nr.tie_sum(first, src, vals).cpu().numpy()
    v = vals.cpu().numpy()
    ref = np.array([sum(v[src[t]] for t in range(first[k], first[k + 1])) for k in range(n_out)])
    assert np.array_equal(out, ref)
