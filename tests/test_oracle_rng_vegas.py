"""Pins for the oracle's random numbers and VEGAS steps (CPU only).

Philox4x64-10 is pinned to numpy's independent implementation of the same
published generator; VEGAS to hand-worked refinement steps and to integrals
with closed forms.
"""
import math

import numpy as np
import pytest

import oracle


def test_philox_matches_numpy_raw_stream():
    # numpy's Philox increments its 256-bit counter before each block, so its
    # k-th block (k = 0, 1, ...) is the raw permutation of counter k + 1.
    for key in ([0, 0], [2105105290, 0], [123456789, 987654321]):
        bg = np.random.Philox(counter=[0, 0, 0, 0], key=key)
        raw = bg.random_raw(4 * 8).reshape(8, 4)
        for k in range(8):
            out = oracle.philox4x64_10([k + 1, 0, 0, 0], key)
            assert np.array_equal(out, raw[k].astype(np.uint64))


def test_philox_carries_into_higher_counter_words():
    key = [7, 11]
    bg = np.random.Philox(counter=np.array([2**64 - 1, 5, 0, 0], dtype=np.uint64), key=key)
    raw = bg.random_raw(4)
    assert np.array_equal(oracle.philox4x64_10([0, 6, 0, 0], key), raw.astype(np.uint64))


def test_uniforms_in_open_interval_and_layout():
    u = oracle.event_uniforms(1000, 13, iteration=3, seed=5, purpose=0)
    assert np.all(u > 0) and np.all(u < 1)
    # event e, call c uses counter (e, iteration, c, 0) and key (seed, purpose)
    o = oracle.philox4x64_10([17, 3, 2, 0], [5, 0])
    expect = ((o >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0**-53
    assert np.array_equal(u[17, 8:12], expect)
    o3 = oracle.philox4x64_10([17, 3, 3, 0], [5, 0])
    assert u[17, 12] == ((int(o3[0]) >> 11) + 0.5) * 2.0**-53
    # different purposes give different streams
    u2 = oracle.event_uniforms(10, 4, iteration=3, seed=5, purpose=1)
    assert not np.allclose(u2, u[:10, :4])
    # mean and variance of a uniform
    big = oracle.event_uniforms(20000, 4, 0, 99)
    assert abs(big.mean() - 0.5) < 5 * math.sqrt(1 / 12 / big.size)


def test_vegas_map_uniform_grid_is_identity():
    e = oracle.uniform_edges(3, 50)
    y = np.array([0.123, 0.5, 0.999])
    x, jac, bins = oracle.vegas_map(e, y)
    assert np.allclose(x, y, atol=1e-15) and abs(jac - 1.0) < 1e-14
    assert list(bins) == [6, 25, 49]


def test_vegas_map_piecewise_linear():
    e = np.array([[0.0, 0.1, 0.5, 1.0]])
    x, jac, bins = oracle.vegas_map(e, np.array([0.5]))  # bin 1 at fraction 0.5
    assert bins[0] == 1 and abs(x[0] - 0.3) < 1e-15 and abs(jac - 3 * 0.4) < 1e-15


def test_refine_hand_worked_single_peak():
    # Five bins, all weight in the middle bin.  Smoothing gives (0, 1/3, 1/3,
    # 1/3, 0); the three non-empty bins get equal importance, so the four new
    # interior edges divide [0.2, 0.8] into five equal shares.
    e = np.linspace(0, 1, 6)[None, :]
    h = np.array([[0.0, 0.0, 1.0, 0.0, 0.0]])
    new = oracle.vegas_refine(e, h, 1.5)
    assert np.allclose(new[0], [0.0, 0.32, 0.44, 0.56, 0.68, 1.0], atol=1e-15)


def test_refine_flat_and_empty_keep_grid():
    e = oracle.uniform_edges(2, 50)
    assert np.allclose(oracle.vegas_refine(e, np.ones((2, 50))), e, atol=1e-15)
    assert np.array_equal(oracle.vegas_refine(e, np.zeros((2, 50))), e)


def test_vegas_constant_integrand():
    e = oracle.uniform_edges(4, 50)
    S1, S2, hist = oracle.vegas_iteration_gauss(4, 0.0, e, 0, 5000, 1)
    assert abs(S1 / 5000 - 1) < 1e-13
    I, s = oracle.iteration_estimate(S1, S2, 5000)
    assert s < 1e-6
    # a flat integrand only moves the edges by counting noise
    assert np.max(np.abs(oracle.vegas_refine(e, hist) - e)) < 0.02


def test_vegas_gaussian_product_closed_form():
    d, sig = 4, 0.1
    exact = math.erf(0.5 / (sig * math.sqrt(2))) ** d
    e = oracle.uniform_edges(d, 50)
    Is, ss = [], []
    for it in range(6):
        S1, S2, hist = oracle.vegas_iteration_gauss(d, sig, e, it, 20000, 77)
        I, s = oracle.iteration_estimate(S1, S2, 20000)
        Is.append(I)
        ss.append(s)
        e = oracle.vegas_refine(e, hist)
    mean, err, chi2 = oracle.combine(Is, ss)
    assert abs(mean - exact) < 3 * err
    assert ss[-1] < 0.3 * ss[0]  # adaptation reduces the variance
    widths = np.diff(e[0])
    assert widths[25] < 0.5 * widths[0]  # bins concentrate at the peak


def test_combine_formula():
    mean, err, chi2 = oracle.combine([1.0, 3.0], [1.0, 1.0])
    assert mean == 2.0 and abs(err - 1 / math.sqrt(2)) < 1e-15 and abs(chi2 - 2.0) < 1e-15
