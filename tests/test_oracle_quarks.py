"""Pins of the oracle's two-quark-line matrix elements (CPU only):
q q~ -> t t~ g and q g -> t t~ q.

* Ward identity: with the external gluon's polarisation replaced by its
  momentum the colour- and helicity-summed |M|^2 vanishes; this fixes the
  relative signs and phases of the five diagrams, the three-gluon vertex
  included (a wrong one leaves a term of the size of |M|^2).
* Collinear limits against the closed-form q q~ -> t t~ matrix element (an
  independent code path, pinned by the textbook formula in test_oracle_me):
  with spin- and colour-averaged |M|^2 and 8 pi alpha_s = 2 g^2,
  - q q~ -> t t~ g with the gluon along the incoming quark (momentum
    fraction x kept by the quark):
      <|M_3|^2> -> 2 g^2 / (x 2 p1.k) C_F (1 + x^2)/(1 - x) <|M_2(x p1, p2)|^2>;
  - q g -> t t~ q with the outgoing quark along the incoming gluon (the
    antiquark entering the hard process carries x p2):
      <|M_3|^2> -> 2 g^2 / (x 2 p2.k) T_R (x^2 + (1 - x)^2) <|M_2(p1, x p2)|^2>,
  with averages 1/36 (q q~), 1/96 (q g).  The ratio tends to 1 as the angle
  shrinks; these fix the absolute normalisation of both processes.
* Lorentz invariance; charge conjugation of q q~ -> t t~ g (quark <->
  antiquark together with top <-> antitop).
* The colour matrix of the five diagrams from explicit Gell-Mann matrices
  against values worked out by hand from Tr(t^a t^b) = delta/2 and the
  Casimirs C_F = 4/3, C_A = 3.
"""
import math

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from oracle import colour

MT = 173.0
CF, TR = 4.0 / 3.0, 0.5


def mdot(a, b):
    return a[0] * b[0] - a[1:] @ b[1:]


def boost(p, beta):
    """Boost p by velocity beta (3-vector)."""
    b2 = beta @ beta
    if b2 == 0:
        return p.copy()
    g = 1.0 / math.sqrt(1.0 - b2)
    bp = beta @ p[1:]
    e = g * (p[0] + bp)
    vec = p[1:] + ((g - 1.0) * bp / b2 + g * p[0]) * beta
    return np.concatenate([[e], vec])


def pair_from(P, mt, ct, phi):
    """t, t~ of total momentum P with the top at (cos theta, phi) in P's rest frame."""
    M = math.sqrt(mdot(P, P))
    q = 0.5 * math.sqrt(M * M - 4 * mt * mt)
    st = math.sqrt(1 - ct * ct)
    t = np.array([M / 2, q * st * math.cos(phi), q * st * math.sin(phi), q * ct])
    tb = np.array([M / 2, -t[1], -t[2], -t[3]])
    beta = P[1:] / P[0]
    return boost(t, beta), boost(tb, beta)


def random_5(seed, rs=1200.0):
    """A point of q q~ -> t t~ + one massless parton from the oracle's phase space."""
    x = si.unit_points(64, 7, seed=seed)
    mom, wt = oracle.phase_space(1, x, rs, MT)
    m = mom[np.argmax(wt > 0)]  # (p1, p2, t, tb, k)
    return m


@pytest.mark.parametrize("kind", ["qqg", "qgq"])
@pytest.mark.parametrize("seed", [3, 4, 5])
def test_ward_identity(kind, seed):
    m = random_5(seed)
    full = oracle.me_qq(kind, m, MT)
    ward = oracle.me_qq(kind, m, MT, ward=True)
    E = m[0, 0]
    assert full > 0
    # the momentum has energy ~ E where a polarisation vector has norm 1, so
    # each diagram is ~ |M| E; the colour form of the cancelling diagrams
    # leaves rounding ~ 1e-16 |M|^2 E^2 (a wrong relative sign leaves ~ 1)
    assert abs(ward) < 1e-12 * full * E * E, (ward, full)


@pytest.mark.parametrize("x", [0.4, 0.75])
def test_collinear_limit_qqbar_g(x):
    rs = 1500.0
    E = rs / 2
    p1 = np.array([E, 0, 0, E])
    p2 = np.array([E, 0, 0, -E])
    t0, tb0 = pair_from(x * p1 + p2, MT, 0.3, 0.7)
    born = oracle.me_qqbar(np.array([x * p1, p2, t0, tb0]), MT)
    devs = []
    for th in (1e-2, 1e-3, 1e-4):
        k = (1 - x) * E * np.array([1, math.sin(th) * math.cos(1.1), math.sin(th) * math.sin(1.1), math.cos(th)])
        t, tb = pair_from(p1 + p2 - k, MT, 0.3, 0.7)
        m3 = oracle.me_qq("qqg", np.array([p1, p2, t, tb, k]), MT)
        limit = 2.0 * CF * (1 + x * x) / (1 - x) / (x * 2 * mdot(p1, k)) * born
        devs.append(abs(m3 / limit - 1))
    assert devs[2] < 1e-3 and devs[2] < devs[1] < devs[0], devs


@pytest.mark.parametrize("x", [0.4, 0.75])
def test_collinear_limit_qg_q(x):
    rs = 1500.0
    E = rs / 2
    p1 = np.array([E, 0, 0, E])
    p2 = np.array([E, 0, 0, -E])
    t0, tb0 = pair_from(p1 + x * p2, MT, -0.4, 2.1)
    born = oracle.me_qqbar(np.array([p1, x * p2, t0, tb0]), MT)
    devs = []
    for th in (1e-2, 1e-3, 1e-4):
        k = (1 - x) * E * np.array([1, math.sin(th) * math.cos(0.4), math.sin(th) * math.sin(0.4), -math.cos(th)])
        t, tb = pair_from(p1 + p2 - k, MT, -0.4, 2.1)
        m3 = oracle.me_qq("qgq", np.array([p1, p2, t, tb, k]), MT)
        limit = 2.0 * TR * (x * x + (1 - x) ** 2) / (x * 2 * mdot(p2, k)) * born * 96.0 / 36.0
        devs.append(abs(m3 / limit - 1))
    assert devs[2] < 1e-3 and devs[2] < devs[1] < devs[0], devs


@pytest.mark.parametrize("kind", ["qqg", "qgq"])
def test_lorentz_invariance(kind):
    m = random_5(7)
    L = si.boost_matrix(np.array([0.2, -0.3, 0.5])) @ si.rotation_matrix(13)
    a = oracle.me_qq(kind, m, MT)
    b = oracle.me_qq(kind, m @ L.T, MT)
    assert abs(b / a - 1) < 1e-11


def test_charge_conjugation_qqbar_g():
    m = random_5(8)
    a = oracle.me_qq("qqg", m, MT)
    c = oracle.me_qq("qqg", m[[1, 0, 3, 2, 4]], MT)
    assert abs(c / a - 1) < 1e-12


def test_colour_matrix_by_hand():
    CC = colour.two_line_colour_matrix()
    assert np.allclose(CC, np.conj(CC.T), atol=1e-13)
    # |C_0|^2 = sum Tr(t^b t^a t^a t^c) Tr(t^b t^c) = (1/2) C_F sum_b Tr(t^b t^b)
    #         = (1/2)(4/3)(4) = 8/3 (the same for d = 1..3);
    # |C_4|^2 = sum f^{abc} f^{ab'c'} Tr(t^b t^b') Tr(t^c t^c') = N_A C_A / 4 = 6
    assert np.allclose(np.diag(CC).real, [8 / 3] * 4 + [6.0], atol=1e-12)
    # C_0 C_1^* = sum Tr(t^b t^a t^c t^a) Tr(t^b t^c) = (1/2) sum Tr(t^a t^b t^a t^b)
    #           = (1/2)(C_F - C_A/2) C_F N = -1/3
    assert abs(CC[0, 1] - (-1.0 / 3.0)) < 1e-12
    # C_0 C_2^* = sum Tr(t^b t^a t^c) Tr(t^b t^c t^a); the Fierz identity
    # sum_b Tr(X t^b) Tr(Y t^b) = (Tr(XY) - Tr X Tr Y / N)/2 gives
    # (C_F^2 N - 2/N)/2 = (16/3 - 2/3)/2 = 7/3
    assert abs(CC[0, 2] - 7.0 / 3.0) < 1e-12
    # C_0 C_4^* = (1/2) sum f^{ade} Tr(t^e t^a t^d) = (1/2)(i/4) f^{ade} f^{ade}
    # = 3i; the other three follow by the antisymmetry of f
    assert np.allclose(CC[:4, 4], [3j, -3j, 3j, -3j], atol=1e-12)
    assert np.min(np.linalg.eigvalsh(CC)) > -1e-12


def test_oracle_quark_channels_integrand_structure():
    """The hadronic integrands of the new channels: finite, zero exactly for
    the events that fail threshold or cuts, non-zero for those that pass, and
    negative only where an interpolated PDF undershoots zero near x = 1 (a
    tiny fraction of the largest weight)."""
    x = si.points_above_threshold(300, 7, 13000.0, MT, seed=17)
    for ch in ("uu~", "dd~", "qg"):
        orc = oracle.Oracle(oracle.Config(n_g=1, channel=ch))
        w, ok = orc.integrand(x, return_pass=True)
        assert np.all(np.isfinite(w)) and np.all(w[~ok] == 0.0) and np.all(w[ok] != 0.0)
        assert np.all(w > -1e-4 * np.max(w)), ch
