"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

Holds none of the integrand's arithmetic: only numpy random draws of points in
the unit hypercube and of generic test momenta, so that the HIP path and the
oracle can be fed identical inputs.
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 2105105290


def ndim(n_final_gluons: int) -> int:
    """Integration dimensions for g g -> t t~ + n gluons: 3 n_final - 2."""
    return 3 * (n_final_gluons + 2) - 2


def unit_points(n: int, d: int, seed: int = BASE_SEED, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """n points uniformly in (lo, hi)^d, float64, row-major [n][d]."""
    rng = np.random.default_rng(seed)
    return lo + (hi - lo) * rng.random((n, d))


def points_above_threshold(n: int, d: int, sqrt_s: float, m_t: float, seed: int = BASE_SEED,
                           margin: float = 1.05) -> np.ndarray:
    """Points whose x1 x2 S exceeds (margin * 2 m_t)^2, so that every event has kinematics."""
    rng = np.random.default_rng(seed)
    out = np.empty((0, d))
    tau_min = (margin * 2 * m_t / sqrt_s) ** 2
    while out.shape[0] < n:
        x = rng.random((2 * n, d))
        x = x[x[:, 0] * x[:, 1] > tau_min]
        out = np.concatenate([out, x])
    return np.ascontiguousarray(out[:n])


def edge_points(d: int) -> np.ndarray:
    """Uniforms at the extremes of (0, 1): the smallest and largest values a Philox draw can give."""
    lo = 0.5 * 2.0**-53
    hi = 1.0 - 0.5 * 2.0**-53
    rows = [np.full(d, 0.5), np.full(d, lo), np.full(d, hi)]
    mix = np.full(d, 0.5)
    mix[0] = mix[1] = hi
    mix[2:] = lo
    rows.append(mix)
    mix2 = np.full(d, hi)
    mix2[2:] = 0.5
    rows.append(mix2)
    return np.array(rows)


def random_grid(d: int, nb: int = 50, seed: int = BASE_SEED, spread: float = 0.9) -> np.ndarray:
    """A strictly increasing random VEGAS grid on [0, 1] per dimension, shape [d][nb+1]."""
    rng = np.random.default_rng(seed)
    w = 1.0 - spread + spread * rng.random((d, nb)) * 2
    e = np.concatenate([np.zeros((d, 1)), np.cumsum(w, axis=1)], axis=1)
    e /= e[:, -1:]
    e[:, -1] = 1.0
    return e


def boost_matrix(beta: np.ndarray) -> np.ndarray:
    """4x4 Lorentz boost with velocity vector beta (|beta| < 1)."""
    b2 = float(beta @ beta)
    g = 1.0 / np.sqrt(1.0 - b2)
    L = np.eye(4)
    L[0, 0] = g
    L[0, 1:] = L[1:, 0] = g * beta
    L[1:, 1:] += (g - 1.0) * np.outer(beta, beta) / b2
    return L


def rotation_matrix(seed: int = BASE_SEED) -> np.ndarray:
    """A random 4x4 spatial rotation."""
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q *= np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    L = np.eye(4)
    L[1:, 1:] = q
    return L


def flow_params(shapes, seed: int = BASE_SEED, scale_out: float = 0.3):
    """Random dense-layer parameters for the coupling flow, one dict per layer.

    shapes: list of (d_in, hidden, d_out) per layer.  Hidden layers use the
    uniform fan-in scaling sqrt(6/fan_in); the output layer is scaled by
    scale_out (0 gives the identity flow).  float64, row-major [in][out].
    """
    rng = np.random.default_rng(seed)
    out = []
    for d_in, h, d_out in shapes:
        a1 = np.sqrt(6.0 / d_in)
        a2 = np.sqrt(6.0 / h)
        out.append({
            "W1": rng.uniform(-a1, a1, (d_in, h)), "b1": rng.uniform(-0.1, 0.1, h),
            "W2": rng.uniform(-a2, a2, (h, h)), "b2": rng.uniform(-0.1, 0.1, h),
            "W3": scale_out * rng.uniform(-a2, a2, (h, d_out)), "b3": scale_out * rng.uniform(-0.5, 0.5, d_out),
        })
    return out


def flow_params_dyadic(shapes, seed: int = BASE_SEED):
    """Coupling-flow parameters whose forward pass is exact in BF16 on inputs
    on the grid (k + 1/2)/16: first-layer weights in {0, 1/4} and biases in
    (0, 1/2] on a 1/128 grid (so every first hidden value is positive with at
    most 8 significant bits), one weight of 1/2 or 1 per second-layer column
    and zero second-layer biases, sparse output weights in {0, +-1/8, +-1/4}
    and output biases on a 1/16 grid.  shapes as for flow_params."""
    rng = np.random.default_rng(seed)
    out = []
    for d_in, h, d_out in shapes:
        W2 = np.zeros((h, h))
        W2[rng.integers(0, h, h), np.arange(h)] = rng.choice([0.5, 1.0], h)
        out.append({
            "W1": rng.integers(0, 2, (d_in, h)) / 4.0, "b1": rng.integers(1, 65, h) / 128.0,
            "W2": W2, "b2": np.zeros(h),
            "W3": rng.integers(-2, 3, (h, d_out)) / 8.0 * (rng.random((h, d_out)) < 0.05),
            "b3": rng.integers(-16, 17, d_out) / 16.0,
        })
    return out


def grid_points(n: int, d: int, cells: int = 16, seed: int = BASE_SEED) -> np.ndarray:
    """[n][d] points at the cell centres (k + 1/2)/cells."""
    return (np.floor(unit_points(n, d, seed=seed) * cells) + 0.5) / cells
