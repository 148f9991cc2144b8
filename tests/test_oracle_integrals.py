"""Integrated pins of the oracle: VEGAS over the full integrand against a
deterministic quadrature of the closed-form partonic cross sections, and the
oracle's dual-number gradients against finite differences and exact scalings."""
import math

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from oracle import quad


@pytest.fixture(scope="module")
def c1():
    return oracle.Oracle(oracle.Config(n_g=0))


def test_quadrature_values(c1):
    # interpolated grid vs analytic PDF differ only by the interpolation error
    a = quad.hadronic_sigma(c1, "gg", analytic_pdf=True)
    b = quad.hadronic_sigma(c1, "gg")
    assert abs(b / a - 1) < 1e-5
    assert 1900 < b < 2000


def test_vegas_gg_ttbar_matches_quadrature(c1):
    ref = quad.hadronic_sigma(c1, "gg")
    mean, err, chi2, _, _ = oracle.vegas_run(c1, 5, 100000, si.BASE_SEED, purpose=2)
    assert abs(mean - ref) < 3 * err
    assert err / mean < 5e-3


def test_vegas_quark_channels_match_quadrature():
    ou = oracle.Oracle(oracle.Config(n_g=0, channel="uu~"))
    od = oracle.Oracle(oracle.Config(n_g=0, channel="dd~"))
    ref = quad.hadronic_sigma(ou, "qq")
    mu, eu, _, _, _ = oracle.vegas_run(ou, 5, 60000, si.BASE_SEED + 1, purpose=2)
    md, ed, _, _, _ = oracle.vegas_run(od, 5, 60000, si.BASE_SEED + 2, purpose=2)
    assert abs(mu + md - ref) < 3 * math.hypot(eu, ed)


def test_gradient_pdf_normalisation_scaling():
    o = oracle.Oracle(oracle.Config(n_g=1))
    x = si.points_above_threshold(300, 7, 13000.0, 173.0, seed=3)
    w, dA = o.integrand_grad(x, 2)
    nz = w != 0
    assert nz.sum() > 100
    assert np.allclose(dA[nz], 2 * w[nz] / 1.6, rtol=1e-13)
    for d in (7, 8, 9):  # quark normalisations do not enter g g processes
        _, dq = o.integrand_grad(x, d)
        assert np.all(dq == 0)
    oq = oracle.Oracle(oracle.Config(n_g=0, channel="uu~"))
    x4 = si.points_above_threshold(200, 4, 13000.0, 173.0, seed=4)
    w, dAu = oq.integrand_grad(x4, 7)
    _, dAg = oq.integrand_grad(x4, 2)
    assert np.all(dAg == 0) and np.any(dAu != 0)


@pytest.mark.parametrize("direction", [1, 3, 4, 5, 6])
def test_gradient_matches_central_differences(direction):
    cfg = oracle.Config(n_g=1)
    o = oracle.Oracle(cfg)
    x = si.points_above_threshold(40, 7, 13000.0, 173.0, seed=5)
    w, dw = o.integrand_grad(x, direction)
    if direction == 1:
        h = 0.05
        plus = oracle.Config(n_g=1, m_t=173.0 + h)
        minus = oracle.Config(n_g=1, m_t=173.0 - h)
    else:
        k = direction - 2
        p = oracle.default_pdf()
        h = 1e-4 * abs(p[k])
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        plus = oracle.Config(n_g=1, pdf=pp)
        minus = oracle.Config(n_g=1, pdf=pm)
    fp = oracle.Oracle(plus).integrand(x)
    fm = oracle.Oracle(minus).integrand(x)
    both = (fp != 0) & (fm != 0) & (w != 0)  # drop events whose threshold status flips
    fd = (fp - fm) / (2 * h)
    scale = np.max(np.abs(dw[both]))
    assert np.max(np.abs(dw[both] - fd[both])) < 1e-5 * scale


def test_mt_derivative_of_cross_section_two_to_two(c1):
    # d sigma / d m_t of g g -> t t~ (mu = m_t): quadrature difference quotient
    # versus the mean pathwise derivative over uniform points.
    h = 0.5
    sp = quad.hadronic_sigma(oracle.Oracle(oracle.Config(n_g=0, m_t=173.0 + h)), "gg")
    sm = quad.hadronic_sigma(oracle.Oracle(oracle.Config(n_g=0, m_t=173.0 - h)), "gg")
    ref = (sp - sm) / (2 * h)
    x = si.unit_points(300000, 4, seed=6)
    _, dw = c1.integrand_grad(x, 1)
    est = dw.mean()
    err = dw.std() / math.sqrt(dw.size)
    assert abs(est - ref) < 4 * err + 1e-3 * abs(ref)
    assert -45 < ref < -38
