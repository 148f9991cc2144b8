"""Pins for the oracle's fiducial cuts (CPU only).

Hand-built events just inside and just outside each edge of the cut
definition: gluon transverse momentum above 20 GeV, lab-frame pseudorapidity
|eta| < 2.5, pairwise Delta R > 0.4 with the azimuthal difference wrapped into
[-pi, pi], all strict.  The lab frame moves along +z with rapidity
y = ln(x1/x2)/2 relative to the partonic frame (parton 1 carries the fraction
x1 of the beam along +z), so a massless gluon's lab pseudorapidity is its
partonic one plus y; the events with x1 != x2 fix the direction of that boost.
The expected decisions come from these definitions, not from the oracle.
"""
import math

import numpy as np
import pytest

import oracle

EPS = 1e-7


def gluon(pt, eta, phi):
    """Massless partonic-frame momentum with the given pT, pseudorapidity and azimuth."""
    return [pt * math.cosh(eta), pt * math.cos(phi), pt * math.sin(phi), pt * math.sinh(eta)]


@pytest.fixture(scope="module")
def c2():
    return oracle.Oracle(oracle.Config(n_g=1))


@pytest.fixture(scope="module")
def c3():
    return oracle.Oracle(oracle.Config(n_g=2, dr_min=0.4))


@pytest.fixture(scope="module")
def c3_nodr():
    return oracle.Oracle(oracle.Config(n_g=2))


def test_pt_edge(c2):
    for eta in (0.0, 1.3, -2.2):
        assert c2.pass_cuts(gluon(20.0 * (1 + EPS), eta, 0.4), 0.1, 0.1)
        assert not c2.pass_cuts(gluon(20.0 * (1 - EPS), eta, 0.4), 0.1, 0.1)
    assert not c2.pass_cuts(gluon(20.0, 0.0, 0.4), 0.1, 0.1)  # strict inequality
    # pT is the transverse part only: a large longitudinal momentum does not help
    assert not c2.pass_cuts(gluon(19.0, 2.4, 1.0), 0.1, 0.1)


def test_eta_edge_without_boost(c2):
    for sign in (1.0, -1.0):
        assert c2.pass_cuts(gluon(50.0, sign * (2.5 - EPS), 2.0), 0.3, 0.3)
        assert not c2.pass_cuts(gluon(50.0, sign * (2.5 + EPS), 2.0), 0.3, 0.3)


def test_eta_is_taken_in_the_lab_frame(c2):
    y = 0.6
    x1, x2 = 0.2, 0.2 * math.exp(-2 * y)  # x1 > x2: the lab frame sees the system move to +z
    # partonic eta +2.0 -> lab +2.6 (fails); -2.0 -> lab -1.4 (passes)
    assert not c2.pass_cuts(gluon(40.0, 2.0, 0.1), x1, x2)
    assert c2.pass_cuts(gluon(40.0, -2.0, 0.1), x1, x2)
    # partonic eta -2.9 would fail in the partonic frame; in the lab it is -2.3
    assert c2.pass_cuts(gluon(40.0, -2.9, 0.1), x1, x2)
    # the mirrored beam configuration moves the other way
    assert c2.pass_cuts(gluon(40.0, 2.0, 0.1), x2, x1)
    assert not c2.pass_cuts(gluon(40.0, -2.0, 0.1), x2, x1)
    assert c2.pass_cuts(gluon(40.0, 2.9, 0.1), x2, x1)
    # just inside / outside the lab edge: partonic eta 2.5 - y -+ EPS
    assert c2.pass_cuts(gluon(40.0, 2.5 - y - EPS, 0.1), x1, x2)
    assert not c2.pass_cuts(gluon(40.0, 2.5 - y + EPS, 0.1), x1, x2)
    assert c2.pass_cuts(gluon(40.0, -2.5 - y + EPS, 0.1), x1, x2)
    assert not c2.pass_cuts(gluon(40.0, -2.5 - y - EPS, 0.1), x1, x2)


@pytest.mark.parametrize("deta_frac", [0.0, 0.6, 1.0])
def test_delta_r_edge(c3, deta_frac):
    # Delta R = 0.4 split between Delta eta and Delta phi
    deta = 0.4 * deta_frac
    dphi = math.sqrt(max(0.4**2 - deta**2, 0.0))
    for scale, expect in ((1 + EPS, True), (1 - EPS, False)):
        g = [gluon(60.0, 0.1, 0.3), gluon(45.0, 0.1 + scale * deta, 0.3 + scale * dphi)]
        assert c3.pass_cuts(np.array(g), 0.15, 0.15) is expect


def test_delta_r_uses_lab_eta_differences(c3):
    # rapidity differences are boost invariant: the same pair passes / fails
    # identically for any x1/x2, as long as both gluons stay inside |eta| < 2.5
    g_close = np.array([gluon(60.0, 0.2, 1.0), gluon(45.0, 0.2 + 0.39, 1.0)])
    g_far = np.array([gluon(60.0, 0.2, 1.0), gluon(45.0, 0.2 + 0.41, 1.0)])
    for x1, x2 in ((0.1, 0.1), (0.2, 0.1), (0.05, 0.2)):
        assert not c3.pass_cuts(g_close, x1, x2)
        assert c3.pass_cuts(g_far, x1, x2)


def test_delta_phi_wraps_across_pi(c3):
    pi = math.pi
    # azimuths pi - 0.1 and -pi + 0.1 are 0.2 apart, not 2 pi - 0.2
    assert not c3.pass_cuts(np.array([gluon(50.0, 0.5, pi - 0.1), gluon(50.0, 0.5, -pi + 0.1)]), 0.1, 0.1)
    assert c3.pass_cuts(np.array([gluon(50.0, 0.5, pi - 0.25), gluon(50.0, 0.5, -pi + 0.25)]), 0.1, 0.1)
    # with a rapidity difference: sqrt(0.30^2 + 0.25^2) = 0.39 fails, sqrt(0.32^2 + 0.25^2) = 0.406 passes
    assert not c3.pass_cuts(np.array([gluon(50.0, 0.5, pi - 0.15), gluon(50.0, 0.8, -pi + 0.1)]), 0.1, 0.1)
    assert c3.pass_cuts(np.array([gluon(50.0, 0.5, pi - 0.15), gluon(50.0, 0.82, -pi + 0.1)]), 0.1, 0.1)
    # the same across zero azimuth, where no wrap is needed
    assert not c3.pass_cuts(np.array([gluon(50.0, 0.5, 0.1), gluon(50.0, 0.5, -0.1)]), 0.1, 0.1)
    assert c3.pass_cuts(np.array([gluon(50.0, 0.5, 0.25), gluon(50.0, 0.5, -0.25)]), 0.1, 0.1)


def test_no_delta_r_cut_without_dr_min(c3_nodr):
    g = np.array([gluon(50.0, 0.5, 1.0), gluon(50.0, 0.51, 1.01)])
    assert c3_nodr.pass_cuts(g, 0.1, 0.1)


def test_every_gluon_is_cut(c3):
    good = gluon(50.0, 0.0, 0.0)
    assert c3.pass_cuts(np.array([good, gluon(50.0, 1.0, 2.0)]), 0.1, 0.1)
    assert not c3.pass_cuts(np.array([good, gluon(19.9, 1.0, 2.0)]), 0.1, 0.1)
    assert not c3.pass_cuts(np.array([gluon(19.9, 1.0, 2.0), good]), 0.1, 0.1)
    assert not c3.pass_cuts(np.array([good, gluon(50.0, 2.6, 2.0)]), 0.1, 0.1)
    assert not c3.pass_cuts(np.array([gluon(50.0, -2.6, 2.0), good]), 0.1, 0.1)


def test_integrand_zero_exactly_when_cut_fails():
    # the integrand applies this decision: events whose gluons fail it weigh 0
    import seeded_inputs as si

    orc = oracle.Oracle(oracle.Config(n_g=2, dr_min=0.4))
    x = si.points_above_threshold(400, 10, 13000.0, 173.0, seed=7)
    w, mom = orc.integrand_momenta(x)
    # momenta are (p1, p2, t, tb, g1, g2); the lab boost comes from x1, x2
    for i in range(x.shape[0]):
        if not np.all(np.isfinite(mom[i])) or mom[i, 2, 0] == 0.0:
            continue
        passed = orc.pass_cuts(mom[i, 4:], x[i, 0], x[i, 1])
        assert (w[i] != 0.0) == passed
