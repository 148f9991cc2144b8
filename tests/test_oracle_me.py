"""Pins for the oracle's matrix elements and colour algebra (CPU only).

Independent references: textbook closed forms (g g, q q~ -> t t~), an
explicit-colour recursion with the full Feynman rules, the Fierz identity in
exact rational arithmetic, gauge invariance (Ward identities), Lorentz
invariance, Bose and charge-conjugation symmetry.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from oracle import colour, quad

MT = 173.0


def _two_body(rs, ct, phi=0.7, mt=MT):
    E = rs / 2
    q = E * math.sqrt(1 - 4 * mt * mt / rs**2)
    st = math.sqrt(1 - ct * ct)
    t = [E, q * st * math.cos(phi), q * st * math.sin(phi), q * ct]
    return np.array([[E, 0, 0, E], [E, 0, 0, -E], t, [E, -t[1], -t[2], -t[3]]], float)


def _mdot(a, b):
    return a[0] * b[0] - a[1:] @ b[1:]


def _kin(ng, rs, seed):
    """First point of a seeded stream that lies above the t t~ threshold."""
    x = si.unit_points(64, si.ndim(ng), seed=seed)
    mom, wt = oracle.phase_space(ng, x, rs, MT)
    return mom[np.argmax(wt > 0)]


@pytest.mark.parametrize("rs,ct", [(500.0, 0.3), (400.0, -0.8), (2000.0, 0.95), (13000.0, 0.0)])
def test_gg_and_qq_closed_forms(rs, ct):
    g4 = (4 * math.pi * 0.118) ** 2
    mom = _two_body(rs, ct)
    s = rs * rs
    t1 = 2 * _mdot(mom[0], mom[2]) / s
    t2 = 2 * _mdot(mom[1], mom[2]) / s
    gg = oracle.me_gg(2, mom, MT) * g4 / 256
    qq = oracle.me_qqbar(mom, MT) * g4 / 36
    assert abs(gg / quad.me_gg_closed(s, t1, t2, MT) - 1) < 1e-12
    assert abs(qq / quad.me_qq_closed(s, t1, t2, MT) - 1) < 1e-12


def test_gg_worked_example_value():
    # sqrt(s) = 500 GeV, cos(theta) = 0.3, alpha_s = 0.118, m_t = 173: the
    # textbook formula evaluated by hand gives 0.543448451554 (g g) and
    # 0.745519882182 (q q~); see tests/golden/closed_form_2to2.txt.
    g4 = (4 * math.pi * 0.118) ** 2
    mom = _two_body(500.0, 0.3)
    assert abs(oracle.me_gg(2, mom, MT) * g4 / 256 - 0.543448451554) < 1e-11
    assert abs(oracle.me_qqbar(mom, MT) * g4 / 36 - 0.745519882182) < 1e-11


def test_partonic_cross_section_is_angular_integral_of_me():
    # d sigma / d cos = beta <|M|^2> / (32 pi s); integrate over cos(theta)
    rs = 700.0
    s = rs * rs
    beta = math.sqrt(1 - 4 * MT * MT / s)
    xs, ws = np.polynomial.legendre.leggauss(60)
    g4 = (4 * math.pi * 0.118) ** 2
    tot_gg = sum(w * oracle.me_gg(2, _two_body(rs, c), MT) * g4 / 256 for c, w in zip(xs, ws))
    tot_qq = sum(w * oracle.me_qqbar(_two_body(rs, c), MT) * g4 / 36 for c, w in zip(xs, ws))
    f = beta / (32 * math.pi * s)
    assert abs(tot_gg * f / quad.sigma_hat_gg(np.array([s]), MT)[0] - 1) < 1e-12
    assert abs(tot_qq * f / quad.sigma_hat_qq(np.array([s]), MT)[0] - 1) < 1e-12


def test_explicit_colour_two_gluons():
    mom = _kin(0, 900.0, 21)
    assert abs(colour.dressed_me(2, mom, MT) / oracle.me_gg(2, mom, MT) - 1) < 1e-12


def test_explicit_colour_three_gluons_per_helicity():
    mom = _kin(1, 1500.0, 22)
    tot, per = oracle.me_gg(3, mom, MT, per_helicity=True)
    hels = [0, 5, 19, 31]
    d = colour.dressed_me(3, mom, MT, helicities=hels)
    assert np.allclose(d, per[hels], rtol=1e-12, atol=1e-14 * tot)


def _fierz_trace(word):
    """Sum over repeated adjoint labels of Tr(t^{w1} ... t^{wk}), exactly (N = 3).

    Uses Tr(X t^a Y t^a) = (Tr X Tr Y - Tr(XY)/N)/2 and
    Tr(X t^a) Tr(Y t^a) = (Tr(XY) - Tr X Tr Y / N)/2 on a product of traces.
    """
    N = Fraction(3)

    def reduce(traces):
        traces = [tuple(t) for t in traces]
        labels = {}
        for ti, t in enumerate(traces):
            for pi, a in enumerate(t):
                labels.setdefault(a, []).append((ti, pi))
        if not labels:
            return N ** len(traces)
        a, ((t1, p1), (t2, p2)) = next(iter(labels.items()))
        if t1 == t2:
            t = traces[t1]
            X, Y, Z = t[:p1], t[p1 + 1:p2], t[p2 + 1:]
            rest = [traces[i] for i in range(len(traces)) if i != t1]
            return Fraction(1, 2) * (reduce(rest + [Z + X, Y]) - reduce(rest + [Z + X + Y]) / N)
        A, B = traces[t1], traces[t2]
        X = A[p1 + 1:] + A[:p1]  # Tr(X t^a) with X the cyclic rest of A
        Y = B[p2 + 1:] + B[:p2]
        rest = [traces[i] for i in range(len(traces)) if i not in (t1, t2)]
        return Fraction(1, 2) * (reduce(rest + [X + Y]) - reduce(rest + [X, Y]) / N)

    return reduce([word])


@pytest.mark.parametrize("m", [2, 3, 4])
def test_colour_matrix_exact_by_fierz(m):
    C = colour.colour_matrix(m)
    perms = list(itertools.permutations(range(m)))
    rows = range(len(perms)) if m < 4 else (0, 7, 23)
    for i in rows:
        for j, sp in enumerate(perms):
            exact = _fierz_trace(tuple(reversed(perms[i])) + sp)
            assert abs(C[i, j] - float(exact)) < 1e-12


@pytest.mark.parametrize("m,den", [(2, 3), (3, 9), (4, 54), (5, 324)])
def test_colour_matrix_structure(m, den):
    C = colour.colour_matrix(m)
    assert np.allclose(C, C.T, atol=1e-12)
    assert np.allclose(np.diag(C), 3 * (4 / 3) ** m, rtol=1e-12)
    z = C * den
    assert np.max(np.abs(z - np.round(z))) < 1e-9
    assert np.min(np.linalg.eigvalsh(C)) > 1.0
    rs = np.sort(C, axis=1)
    assert np.allclose(rs, rs[0], atol=1e-12)  # rows are permutations of each other


@pytest.mark.parametrize("m", [2, 3, 4])
def test_colour_relabelling_identity(m):
    assert np.allclose(colour.colour_matrix_by_relabelling(m), colour.colour_matrix(m), atol=1e-12)


@pytest.mark.parametrize("m,rs,seed", [(3, 1500.0, 31), (4, 2500.0, 32), (5, 3500.0, 33)])
def test_ward_identity_every_partial_amplitude(m, rs, seed):
    mom = _kin(m - 2, rs, seed)
    k = np.concatenate([mom[:2], mom[4:]])
    inc = [1, 1] + [0] * (m - 2)
    for h in (0, 3, (1 << (m + 2)) - 1, 9):
        ref = oracle.partial_amplitudes(m, k, inc, mom[2], mom[3], MT, h)
        scale = np.max(np.abs(ref))
        assert scale > 0
        for g in range(m):
            a = oracle.partial_amplitudes(m, k, inc, mom[2], mom[3], MT, h, ward=g)
            # the momentum has energy ~ rs/2 where a polarisation has norm 1
            assert np.max(np.abs(a)) < 1e-12 * scale * rs


@pytest.mark.parametrize("m,rs", [(2, 800.0), (3, 1500.0), (4, 2500.0)])
def test_lorentz_invariance(m, rs):
    mom = _kin(m - 2, rs, 40 + m)
    L = si.boost_matrix(np.array([0.3, -0.5, 0.2])) @ si.rotation_matrix(7)
    a = oracle.me_gg(m, mom, MT)
    b = oracle.me_gg(m, mom @ L.T, MT)
    assert abs(b / a - 1) < 1e-11


def test_bose_and_charge_conjugation_symmetry():
    mom = _kin(2, 2500.0, 51)
    a = oracle.me_gg(4, mom, MT)
    sw = mom.copy()
    sw[[4, 5]] = sw[[5, 4]]
    assert abs(oracle.me_gg(4, sw, MT) / a - 1) < 1e-12
    sw = mom.copy()
    sw[[0, 1]] = sw[[1, 0]]
    assert abs(oracle.me_gg(4, sw, MT) / a - 1) < 1e-12
    sw = mom.copy()
    sw[[2, 3]] = sw[[3, 2]]
    assert abs(oracle.me_gg(4, sw, MT) / a - 1) < 1e-12
    mom3 = _kin(1, 1500.0, 52)
    sw = mom3.copy()
    sw[[0, 1]] = sw[[1, 0]]
    assert abs(oracle.me_gg(3, sw, MT) / oracle.me_gg(3, mom3, MT) - 1) < 1e-12


def test_spinor_and_polarisation_identities():
    G = oracle.gamma_matrices()
    metric = np.array([1.0, -1, -1, -1])
    sl = lambda p: np.einsum("m,mrc,m->rc", metric, G, p)
    p = np.array([0.0, 30.0, -50.0, 120.0])
    p[0] = math.sqrt(MT**2 + p[1:] @ p[1:])
    sum_uu = sum(np.outer(oracle.wavefunction("u", p, MT, l), oracle.wavefunction("ubar", p, MT, l)) for l in (-1, 1))
    sum_vv = sum(np.outer(oracle.wavefunction("v", p, MT, l), oracle.wavefunction("vbar", p, MT, l)) for l in (-1, 1))
    assert np.allclose(sum_uu, sl(p) + MT * np.eye(4), atol=1e-10)
    assert np.allclose(sum_vv, sl(p) - MT * np.eye(4), atol=1e-10)
    for l in (-1, 1):
        assert np.allclose((sl(p) - MT * np.eye(4)) @ oracle.wavefunction("u", p, MT, l), 0, atol=1e-10)
        assert np.allclose((sl(p) + MT * np.eye(4)) @ oracle.wavefunction("v", p, MT, l), 0, atol=1e-10)
    for k in (np.array([5.0, 3.0, 0.0, 4.0]), np.array([7.0, 0, 0, -7.0]), np.array([2.0, 0, 0, 2.0])):
        e = [oracle.wavefunction("eps", k, 0.0, l) for l in (-1, 1)]
        for v in e:
            assert abs(v[0] * k[0] - v[1:] @ k[1:]) < 1e-14  # transverse
            assert abs((np.conj(v[0]) * v[0] - np.conj(v[1:]) @ v[1:]) + 1) < 1e-14  # eps*.eps = -1
        proj = sum(np.outer(v, np.conj(v)) for v in e)
        kh = k[1:] / k[0]
        assert np.allclose(proj[1:, 1:].real, np.eye(3) - np.outer(kh, kh), atol=1e-14)
