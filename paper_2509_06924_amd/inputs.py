"""Seeded synthetic workloads.

This module only draws inputs: parameter draws, momentum-transfer grids,
resolutions and a synthetic measured curve.  It holds none of the model's
arithmetic; both the HIP path and the CPU oracle consume what it returns.

The paper's datasets (D17 quartz, the OLED devices, the lipid bilayer) are not
available, so every workload is a stand-in with the shapes of the paper's
problems (Sec. 3 parameter dict; Sec. 4 case studies): a fronting medium, L
finite layers and a backing, log-spaced Q grids, constant dQ/Q resolution.
The "measured" curve is a model-free shape with the dynamic range of a
reflectivity curve (about 1 at the lowest Q down to ~1e-7 at the highest, with
fringes), 3 % Gaussian noise and a 1e-7 background.  Likelihood and gradient
values and their cost do not depend on whether the curve is one the model can
fit.

Seeds are numpy.random.default_rng(2509069240 + k) for workload k.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2509069240
SI_SLD = 2.07e-6


@dataclass
class Batch:
    """A batch in the C-ABI layout (host NumPy arrays)."""
    name: str
    q_off: np.ndarray            # int64 [n_datasets + 1]
    Q: np.ndarray                # float64 packed
    Robs: np.ndarray
    Rerr: np.ndarray
    dq_over_q: np.ndarray        # float64 [n_datasets]
    dataset_of_item: np.ndarray  # int32 [n_items]
    row_off: np.ndarray          # int64 [n_items + 1]
    layers: np.ndarray           # float64 [rows, 4]
    scale: np.ndarray            # float64 [n_items]
    bkg: np.ndarray              # float64 [n_items]
    meta: dict = field(default_factory=dict)

    @property
    def n_items(self):
        return int(self.dataset_of_item.size)

    @property
    def n_datasets(self):
        return int(self.dq_over_q.size)

    def rows_of(self, b):
        return self.layers[self.row_off[b]:self.row_off[b + 1]]

    def data_of(self, b):
        s = int(self.dataset_of_item[b])
        a, e = int(self.q_off[s]), int(self.q_off[s + 1])
        return self.Q[a:e], self.Robs[a:e], self.Rerr[a:e], float(self.dq_over_q[s])

    def n_points_of(self, b):
        s = int(self.dataset_of_item[b])
        return int(self.q_off[s + 1] - self.q_off[s])

    def layer_steps(self):
        """Sum over items of nodes x (L+1): the unit of the throughput metric."""
        L = np.diff(self.row_off) - 2
        npts = np.diff(self.q_off)[self.dataset_of_item]
        K = np.where(self.dq_over_q[self.dataset_of_item] > 0, 17, 1)
        return int(np.sum(npts * K * (L + 1)))

    def data_points(self):
        """Sum over items of data points: the secondary unit (draw x Q)."""
        return int(np.sum(np.diff(self.q_off)[self.dataset_of_item]))

    def subset(self, items):
        """A batch of the given items (keeps every dataset)."""
        items = np.asarray(items, dtype=np.int64)
        rows = [self.rows_of(int(b)) for b in items]
        row_off = np.zeros(items.size + 1, np.int64)
        row_off[1:] = np.cumsum([r.shape[0] for r in rows])
        return Batch(self.name + "[subset]", self.q_off.copy(), self.Q, self.Robs,
                     self.Rerr, self.dq_over_q, self.dataset_of_item[items].copy(),
                     row_off, np.vstack(rows) if rows else np.zeros((0, 4)),
                     self.scale[items].copy(), self.bkg[items].copy(), dict(self.meta))


def log_grid(lo, hi, n):
    return np.geomspace(lo, hi, n)


def synthetic_curve(Q, rng, rel_noise=0.03, bkg=1e-7, fringe_period=0.021):
    """Model-free stand-in for a measured curve: smooth power-law decay with
    a shoulder near 0.01 A^-1, sinusoidal fringes, background, 3 % noise."""
    Qk = 0.0102 * 0.7
    base = 1.0 / (1.0 + (Q / Qk) ** 4)
    fr = 1.0 + 0.4 * np.sin(2.0 * np.pi * Q / fringe_period) * (Q > 0.0102)
    R = base * fr + bkg
    err = rel_noise * R
    Robs = R + err * rng.standard_normal(Q.size)
    return Robs, err


def draw_stack(rng, L, d=(10.0, 300.0), rho=(-0.5e-6, 6.5e-6), rho_im=(0.0, 1e-8),
               sigma=(1.0, 15.0), fronting=0.0, backing=SI_SLD):
    rows = np.zeros((L + 2, 4))
    rows[0, 1] = fronting
    rows[1:L + 1, 0] = rng.uniform(*d, L)
    rows[1:L + 1, 1] = rng.uniform(*rho, L)
    rows[1:L + 1, 2] = rng.uniform(*rho_im, L)
    rows[L + 1, 1] = backing
    rows[1:, 3] = rng.uniform(*sigma, L + 1)
    return rows


def _pack(name, datasets, items, meta):
    """datasets: list of (Q, Robs, Rerr, dqq); items: list of (ds, rows, scale, bkg)."""
    q_off = np.zeros(len(datasets) + 1, np.int64)
    q_off[1:] = np.cumsum([d[0].size for d in datasets])
    Q = np.concatenate([d[0] for d in datasets]) if datasets else np.zeros(0)
    Robs = np.concatenate([d[1] for d in datasets]) if datasets else np.zeros(0)
    Rerr = np.concatenate([d[2] for d in datasets]) if datasets else np.zeros(0)
    dqq = np.array([d[3] for d in datasets], np.float64)
    dsi = np.array([it[0] for it in items], np.int32)
    row_off = np.zeros(len(items) + 1, np.int64)
    row_off[1:] = np.cumsum([it[1].shape[0] for it in items])
    layers = np.vstack([it[1] for it in items]) if items else np.zeros((0, 4))
    scale = np.array([it[2] for it in items], np.float64)
    bkg = np.array([it[3] for it in items], np.float64)
    return Batch(name, q_off, Q, Robs, Rerr, dqq, dsi, row_off,
                 np.ascontiguousarray(layers), scale, bkg, meta)


def c1_single_film(seed_offset=1, nq=200):
    """One draw of a thick oxide film on Si: 200 log-Q in [0.008, 0.3], no smearing."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    rows = np.zeros((3, 4))
    rows[1, 0] = rng.uniform(500.0, 1500.0)
    rows[1, 1] = 3.47e-6
    rows[1, 3] = rng.uniform(2.0, 10.0)
    rows[2, 1] = SI_SLD
    rows[2, 3] = rng.uniform(2.0, 8.0)
    Q = log_grid(0.008, 0.3, nq)
    Robs, err = synthetic_curve(Q, rng)
    return _pack("C1 single film, 1 layer, 200 Q, unsmeared", [(Q, Robs, err, 0.0)],
                 [(0, rows, 1.0, 1e-7)], {"config": 1})


def c2_batched(n_items=4096, nq=400, L=10, dq_over_q=0.05, seed_offset=2):
    """4096 draws of a 10-layer stack sharing one 400-point dataset, 5 % dQ/Q."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    Q = log_grid(0.005, 0.35, nq)
    Robs, err = synthetic_curve(Q, rng)
    items = []
    for _ in range(n_items):
        rows = draw_stack(rng, L)
        items.append((0, rows, rng.uniform(0.9, 1.1), rng.uniform(0.5e-7, 1.5e-7)))
    return _pack(f"C2 {n_items} draws x {L} layers x {nq} Q, dQ/Q {dq_over_q:g}",
                 [(Q, Robs, err, dq_over_q)], items, {"config": 2, "L": L, "nq": nq})


def c3_cofit(n_draws=1024, nqs=(250, 300, 350), L=12, dq_over_q=0.05, seed_offset=3):
    """OLED-like co-fit: one 12-layer draw under 3 contrasts (backing SLD
    2.07e-6 / 4.0e-6 / 6.35e-6), uneven Q grids; items draw-major."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    backs = (2.07e-6, 4.0e-6, 6.35e-6)
    datasets = []
    for nq in nqs:
        Q = log_grid(0.005, 0.35, nq)
        Robs, err = synthetic_curve(Q, rng)
        datasets.append((Q, Robs, err, dq_over_q))
    items = []
    for _ in range(n_draws):
        base = draw_stack(rng, L, d=(20.0, 80.0), rho=(0.5e-6, 4.5e-6), sigma=(2.0, 10.0))
        bkg = rng.uniform(0.5e-7, 1.5e-7)
        for c, back in enumerate(backs):
            rows = base.copy()
            rows[-1, 1] = back
            items.append((c, rows, 1.0, bkg))
    return _pack(f"C3 {n_draws} draws x 3 contrasts x {L} layers, Q {'/'.join(map(str, nqs))}",
                 datasets, items, {"config": 3, "L": L, "contrasts": 3})


def c4_ragged(n_items=16384, L_range=(2, 40), nq_range=(100, 1000), dqq_range=(0.02, 0.08),
              seed_offset=4):
    """Independent datasets with uneven layer counts and Q lengths."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    datasets, items = [], []
    for b in range(n_items):
        L = int(rng.integers(L_range[0], L_range[1] + 1))
        nq = int(rng.integers(nq_range[0], nq_range[1] + 1))
        dqq = float(rng.uniform(*dqq_range))
        Q = log_grid(0.005, 0.35, nq)
        Robs, err = synthetic_curve(Q, rng)
        datasets.append((Q, Robs, err, dqq))
        items.append((b, draw_stack(rng, L), rng.uniform(0.9, 1.1), rng.uniform(0.5e-7, 1.5e-7)))
    return _pack(f"C4 {n_items} ragged items, L {L_range}, nQ {nq_range}", datasets, items,
                 {"config": 4})


def c5_vi(n_samples=8192, nq=1000, L=20, dq_over_q=0.05, rel_width=0.01, seed_offset=5):
    """Mean-field VI samples theta = mu + s * eps over a 20-layer stack; the
    standard normal draws eps are returned in meta for the sampler."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    Q = log_grid(0.005, 0.35, nq)
    Robs, err = synthetic_curve(Q, rng)
    mu = draw_stack(rng, L)
    eps = rng.standard_normal((n_samples, L, 4))
    items = []
    for i in range(n_samples):
        rows = mu.copy()
        rows[1:L + 1] = mu[1:L + 1] + rel_width * np.abs(mu[1:L + 1]) * eps[i]
        rows[1:L + 1, 0] = np.abs(rows[1:L + 1, 0])
        items.append((0, rows, 1.0, 1e-7))
    return _pack(f"C5 {n_samples} VI samples x {L} layers x {nq} Q", [(Q, Robs, err, dq_over_q)],
                 items, {"config": 5, "mu": mu, "eps": eps, "rel_width": rel_width})


def microsliced(n_items=64, L=1000, nq=200, dz=2.0, dq_over_q=0.05, seed_offset=6):
    """Microsliced SLD profiles (hundreds to thousands of slabs): each item
    samples a smooth two-film profile on silicon in L slices of dz A (small
    absorption, 0.5 A slice roughness); one dataset of nq log-spaced points."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    Q = log_grid(0.005, 0.3, nq)
    Robs, err = synthetic_curve(Q, rng)
    items = []
    for _ in range(n_items):
        rows = microsliced_stack(rng, L, dz)
        items.append((0, rows, float(rng.uniform(0.9, 1.1)), 1e-7))
    return _pack("microsliced", [(Q, Robs, err, dq_over_q)], items,
                 {"L": L, "dz": dz})


def microsliced_stack(rng, L, dz=2.0):
    """One microsliced profile: L slices of dz A sampling a smooth two-film
    SLD curve (centres at 0.2-0.4 and 0.6-0.8 of the depth, widths 3-8 %)
    on silicon, absorption 5e-8, slice roughness 0.5 A, backing roughness
    3 A."""
    z = (np.arange(L) + 0.5) * dz
    span = L * dz
    c1, c2 = rng.uniform(0.2, 0.4) * span, rng.uniform(0.6, 0.8) * span
    w = rng.uniform(0.03, 0.08) * span
    rows = np.zeros((L + 2, 4))
    rows[1:L + 1, 0] = dz
    rows[1:L + 1, 1] = (1.0e-6 + 3.0e-6 / (1 + np.exp(-(z - c1) / w))
                        - 2.0e-6 / (1 + np.exp(-(z - c2) / w)))
    rows[1:L + 1, 2] = 5e-8
    rows[1:L + 1, 3] = 0.5
    rows[L + 1] = [0.0, SI_SLD, 5e-8, 3.0]
    return rows


def random_batch(rng, n_items, L_choices, nq_choices, dqq_choices, n_datasets=None):
    """Small ragged batch for parity tests (shares datasets between items)."""
    n_datasets = n_datasets or max(1, n_items // 2)
    datasets = []
    for _ in range(n_datasets):
        nq = int(rng.choice(nq_choices))
        Q = log_grid(0.005, 0.35, nq) if nq > 0 else np.zeros(0)
        Robs, err = synthetic_curve(Q, rng)
        datasets.append((Q, Robs, err, float(rng.choice(dqq_choices))))
    items = []
    for _ in range(n_items):
        L = int(rng.choice(L_choices))
        items.append((int(rng.integers(0, n_datasets)), draw_stack(rng, L),
                      rng.uniform(0.9, 1.1), rng.uniform(0.5e-7, 1.5e-7)))
    return _pack("random", datasets, items, {})
