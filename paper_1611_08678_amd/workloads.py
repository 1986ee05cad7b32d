"""Seeded synthetic workloads (inputs only).

This module draws the inputs of the benchmark/parity workloads with
numpy's PCG64 generator and holds no arithmetic of the method itself; the
oracle and the HIP library both take their inputs from here. Each workload is
a dict with keys: system, theta [B, n_params], alpha [B], h [B], N [B],
y0 [B, d] (B = 1 for single trajectories) plus descriptive fields.

  scalar_linear  D^0.5 y = -y, y(0) = 1, h = 0.005, N = 2000 (T = 10)
  chen           Chen (a, b, c) = (35, 3, 28), alpha 0.95, y0 = (-9, -5, 14),
                 h = 0.001, N = 2^20
  rossler_batch  4096 Rossler (0.2, 0.2, 5.7), y0 ~ U[-5, 5]^3,
                 alpha ~ U[0.9, 1.0], N ~ U{2^14 .. 2^17}, h = 0.005 (seed 2);
                 about 2% of these starting points leave every bounded set
                 within a few hundred steps
  linear64_batch 512 linear systems, d = 64, A = -(2 I + G/8), G_ij ~ N(0, 1),
                 y0 ~ N(0, 1), alpha 0.8, h = 0.01, N = 2^16 (seed 3)
  vdp_adjoint    1024 Van der Pol, mu ~ U[0.5, 2], y0 ~ U[-2, 2]^2,
                 target mu_hat = mu + N(0, 0.05^2), alpha 0.9, h = 0.01,
                 N = 2^15 (seed 4)
  hindmarsh_rose Hindmarsh-Rose neuron (a, b, c, d, r, s, xr, I) =
                 (1, 3, 1, 5, 0.006, 4, -1.6, 3.25), alpha 0.95, h = 0.01,
                 y0 = (-1.6, -10, 2); N from the step counts of the paper's
                 Section 4 timing table (TABLE2_N)
  per_component_orders  any of the above with alpha [B][d] ~ U[lo, 1] (seed 6;
                 lo = 0.8, 0.9 for the Rossler batch)
"""
from __future__ import annotations

import numpy as np

LINEAR, CHEN, ROSSLER, VDP, FINANCIAL, HINDMARSH_ROSE = 0, 1, 2, 3, 4, 5


def _linear_theta(A, b0=None, b1=None):
    A = np.asarray(A, dtype=np.float64)
    B, d, _ = A.shape
    b0 = np.zeros((B, d)) if b0 is None else np.asarray(b0, np.float64)
    b1 = np.zeros((B, d)) if b1 is None else np.asarray(b1, np.float64)
    return np.concatenate([A.reshape(B, d * d), b0, b1], axis=1)


def scalar_linear(N: int = 2000, h: float = 0.005):
    return dict(name="scalar_linear", system=LINEAR, d=1,
                theta=_linear_theta(np.full((1, 1, 1), -1.0)), alpha=np.array([0.5]),
                h=np.array([h]), N=np.array([N], dtype=np.int64), y0=np.ones((1, 1)))


def chen(N: int = 1 << 20, h: float = 0.001):
    return dict(name="chen", system=CHEN, d=3, theta=np.array([[35.0, 3.0, 28.0]]),
                alpha=np.array([0.95]), h=np.array([h]), N=np.array([N], dtype=np.int64),
                y0=np.array([[-9.0, -5.0, 14.0]]))


def rossler_batch(batch: int = 4096, n_lo: int = 1 << 14, n_hi: int = 1 << 17, seed: int = 2,
                  h: float = 0.005):
    rng = np.random.Generator(np.random.PCG64(seed))
    y0 = rng.uniform(-5.0, 5.0, size=(batch, 3))
    alpha = rng.uniform(0.9, 1.0, size=batch)
    N = rng.integers(n_lo, n_hi, size=batch, endpoint=True).astype(np.int64)
    return dict(name="rossler_batch", system=ROSSLER, d=3,
                theta=np.tile([0.2, 0.2, 5.7], (batch, 1)), alpha=alpha,
                h=np.full(batch, h), N=N, y0=y0)


def linear64_batch(batch: int = 512, d: int = 64, N: int = 1 << 16, seed: int = 3,
                   h: float = 0.01, alpha: float = 0.8):
    rng = np.random.Generator(np.random.PCG64(seed))
    G = rng.standard_normal((batch, d, d))
    y0 = rng.standard_normal((batch, d))
    A = -(2.0 * np.eye(d)[None, :, :] + G / 8.0)
    return dict(name="linear64_batch", system=LINEAR, d=d, theta=_linear_theta(A),
                alpha=np.full(batch, alpha), h=np.full(batch, h),
                N=np.full(batch, N, dtype=np.int64), y0=y0)


def vdp_adjoint(batch: int = 1024, N: int = 1 << 15, seed: int = 4, h: float = 0.01,
                alpha: float = 0.9):
    rng = np.random.Generator(np.random.PCG64(seed))
    mu = rng.uniform(0.5, 2.0, size=batch)
    y0 = rng.uniform(-2.0, 2.0, size=(batch, 2))
    eps = rng.normal(0.0, 0.05, size=batch)
    return dict(name="vdp_adjoint", system=VDP, d=2, theta=mu[:, None].copy(),
                theta_target=(mu + eps)[:, None].copy(), alpha=np.full(batch, alpha),
                h=np.full(batch, h), N=np.full(batch, N, dtype=np.int64), y0=y0)


# Step counts of the paper's Section 4 comparison of cluster and GPU run times
# (Table 2); the model parameters, alpha and h of those runs are not given.
TABLE2_N = (100_000, 500_000, 1_000_000, 1_500_000, 2_000_000, 2_500_000, 3_000_000)
HR_THETA = (1.0, 3.0, 1.0, 5.0, 0.006, 4.0, -1.6, 3.25)


def hindmarsh_rose(N: int = 1_000_000, h: float = 0.01, alpha: float = 0.95):
    """One Hindmarsh-Rose trajectory in the bursting regime of the integer-order
    model (the parameter set most used in the literature); theta follows the
    layout of the device system (a, b, c, d, r, s, xr, I)."""
    return dict(name="hindmarsh_rose", system=HINDMARSH_ROSE, d=3,
                theta=np.array([HR_THETA]), alpha=np.array([alpha]), h=np.array([h]),
                N=np.array([N], dtype=np.int64), y0=np.array([[-1.6, -10.0, 2.0]]))


def per_component_orders(w: dict, lo: float = 0.8, hi: float = 1.0, seed: int = 6):
    """The same workload with a separate order per state component
    (non-commensurate system): alpha [B][d] uniform in [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    B, d = len(w["N"]), w["d"]
    out = dict(w)
    out["alpha"] = rng.uniform(lo, hi, size=(B, d))
    out["name"] = w["name"] + "_orders"
    return out


def random_history(N: int, d: int, seed: int = 0):
    """A smooth-plus-noise history f_0..f_{N-1} for teacher-forced contraction
    tests (values of order 1 with varying sign)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.arange(N)[:, None] / max(N, 1)
    phase = rng.uniform(0, 2 * np.pi, size=(1, d))
    return np.sin(40.0 * t + phase) + 0.25 * rng.standard_normal((N, d))
