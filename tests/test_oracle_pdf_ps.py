"""Pins for the oracle's PDF interpolation and phase-space generator (CPU only)."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import seeded_inputs as si


@pytest.fixture(scope="module")
def orc():
    return oracle.Oracle(oracle.Config(n_g=0))


def test_pdf_knot_values_exact(orc):
    xk, qk = oracle.x_knots(), oracle.q_knots()
    for fl in oracle.FLAVOURS:
        tab = orc.pdf_table(fl)
        for j in (0, 7, 30, 49):
            v = orc.pdf(fl, xk[:-1], np.full(195, qk[j]))
            assert np.allclose(v, tab[j, :-1], rtol=1e-12, atol=0)
        A, a, b, c, d = oracle.PDF_PARAMS[fl]
        L = math.log(qk[10] / 1.65)
        x = xk[50]
        assert abs(tab[10, 50] / (A * x ** (a + b * L) * (1 - x) ** (c + d * L)) - 1) < 1e-13


def test_interpolant_reproduces_biquadratic():
    # Cubic Hermite with central-difference slopes is exact for quadratics, so
    # the tensor product reproduces (quadratic in ln x) x (quadratic in ln Q)
    # between the second and the next-to-last knots.
    lx = np.log(oracle.x_knots())
    lq = np.log(oracle.q_knots())
    fx = lambda t: 0.3 + 0.2 * t - 0.01 * t * t
    fq = lambda t: 1.1 - 0.4 * t + 0.05 * t * t
    tab = fq(lq)[:, None] * fx(lx)[None, :]
    rng = np.random.default_rng(1)
    x = np.exp(rng.uniform(lx[1], lx[-2], 200))
    Q = np.exp(rng.uniform(lq[1], lq[-2], 200))
    got = oracle.hermite2d(tab, x, Q)
    exact = fq(np.log(Q)) * fx(np.log(x))
    assert np.max(np.abs(got / exact - 1)) < 1e-13


def test_interpolation_error_vs_analytic(orc):
    # Smooth region: the log-bicubic interpolant follows the formula closely.
    for x, tol in ((1e-3, 5e-5), (1e-2, 5e-6), (0.1, 2e-5), (0.3, 3e-4)):
        a = orc.pdf("g", x, 173.0, analytic=True)[0]
        b = orc.pdf("g", x, 173.0)[0]
        assert abs(b / a - 1) < tol


def test_phase_space_conservation_and_mass_shell():
    mt = 173.0
    for ng in (0, 1, 2, 3):
        d = si.ndim(ng)
        x = si.unit_points(300, d, seed=11 + ng)
        mom, wt = oracle.phase_space(ng, x, 1500.0, mt)
        ok = wt > 0
        assert ok.sum() > 100
        p = mom[ok]
        tot_out = p[:, 2:, :].sum(axis=1)
        tot_in = p[:, 0, :] + p[:, 1, :]
        assert np.max(np.abs(tot_out - tot_in)) < 1e-11 * 1500
        m2 = p[..., 0] ** 2 - np.sum(p[..., 1:] ** 2, axis=-1)
        assert np.allclose(m2[:, 2], mt * mt, rtol=1e-10)
        assert np.allclose(m2[:, 3], mt * mt, rtol=1e-10)
        if ng:
            assert np.max(np.abs(m2[:, 4:])) < 1e-9 * 1500**2


def test_massless_weight_is_volume():
    # with m_t = 0 every point carries exactly the massless volume V_n(s)
    for ng, s in ((0, 500.0**2), (1, 1e6), (2, 4e6), (3, 9e6)):
        n = ng + 2
        V = (2 * math.pi) ** (4 - 3 * n) * (math.pi / 2) ** (n - 1) * s ** (n - 2) / (
            math.factorial(n - 1) * math.factorial(n - 2))
        x = si.unit_points(50, si.ndim(ng), seed=5)
        _, wt = oracle.phase_space(ng, x, math.sqrt(s), 0.0)
        assert np.allclose(wt, V, rtol=1e-13)
    assert abs(1 / (8 * math.pi) - (2 * math.pi) ** -2 * (math.pi / 2)) < 1e-16


def test_massless_flatness_by_symmetry():
    # flat massless phase space is symmetric under particle permutations:
    # <x_i> = 2/3 for three bodies (flat Dalitz plot), <s_ij>/s = 1/6 for four.
    mom, _ = oracle.phase_space(1, si.unit_points(200000, 7, seed=3), 1000.0, 0.0)
    xfr = 2 * mom[:, 2:, 0] / 1000.0
    err = np.std(xfr, axis=0) / math.sqrt(xfr.shape[0])
    assert np.all(np.abs(xfr.mean(axis=0) - 2 / 3) < 5 * err)
    mom, _ = oracle.phase_space(2, si.unit_points(200000, 10, seed=4), 1000.0, 0.0)
    fs = mom[:, 2:, :]
    for i in range(4):
        for j in range(i + 1, 4):
            p = fs[:, i] + fs[:, j]
            sij = (p[:, 0] ** 2 - np.sum(p[:, 1:] ** 2, axis=1)) / 1e6
            assert abs(sij.mean() - 1 / 6) < 5 * sij.std() / math.sqrt(sij.size)


def _phi2(M, m1, m2):
    lam = (1 - (m1 + m2) ** 2 / M**2) * (1 - (m1 - m2) ** 2 / M**2)
    return math.sqrt(max(lam, 0.0)) / (8 * math.pi)


def test_massive_volume_against_nested_two_body_integrals():
    mt, rs = 173.0, 1500.0
    # three bodies: int dM^2/2pi Phi2(rs; 0, M) Phi2(M; m, m)
    V3, _ = integrate.quad(lambda M2: _phi2(rs, 0, math.sqrt(M2)) * _phi2(math.sqrt(M2), mt, mt) / (2 * math.pi),
                           4 * mt * mt, rs * rs, epsrel=1e-12)
    _, wt = oracle.phase_space(1, si.unit_points(400000, 7, seed=8), rs, mt)
    assert abs(wt.mean() - V3) < 4 * wt.std() / math.sqrt(wt.size)
    # four bodies
    def inner(M1sq):
        M1 = math.sqrt(M1sq)
        v, _ = integrate.quad(lambda M2: _phi2(M1, 0, math.sqrt(M2)) * _phi2(math.sqrt(M2), mt, mt) / (2 * math.pi),
                              4 * mt * mt, M1sq, epsrel=1e-11)
        return _phi2(rs, 0, M1) * v / (2 * math.pi)
    V4, _ = integrate.quad(inner, 4 * mt * mt, rs * rs, epsrel=1e-10)
    _, wt = oracle.phase_space(2, si.unit_points(400000, 10, seed=9), rs, mt)
    assert abs(wt.mean() - V4) < 4 * wt.std() / math.sqrt(wt.size)


def test_two_body_weight_and_angles():
    mt, rs = 173.0, 500.0
    x = np.array([[0.5, 0.5, 0.65, 0.25]])
    mom, wt = oracle.phase_space(0, x, rs, mt)
    beta = math.sqrt(1 - 4 * mt * mt / rs**2)
    assert abs(wt[0] - beta / (8 * math.pi)) < 1e-16
    t = mom[0, 2]
    q = rs / 2 * beta
    assert abs(t[3] / q - 0.3) < 1e-14  # cos(theta) = 2 x - 1
    assert abs(math.atan2(t[2], t[1]) - 0.5 * math.pi) < 1e-14  # phi = 2 pi x
