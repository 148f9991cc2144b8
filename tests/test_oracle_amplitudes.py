"""Further pins for the oracle's colour-ordered amplitudes (CPU only).

* U(1) decoupling (the Abelian identity): summed over all orderings of the
  gluons along the quark line, the colour-ordered amplitudes of a top pair and
  m gluons equal the amplitude with every gluon replaced by a photon, i.e. the
  fermion line alone with its m! attachment orders and no gluon self-coupling.
  The photon amplitude is written below from the QED Feynman rules, with the
  oracle's wavefunctions and Dirac matrices (pinned in test_oracle_me) as its
  only inputs; the three- and four-gluon vertices drop out of the sum only if
  their signs and normalisations are right.
* Massless limit (Parke-Taylor / Mangano-Parke): with m_t = 0, a partial
  amplitude of a quark pair and m gluons in which exactly two particles
  (counted as outgoing) have negative helicity, or exactly two positive, has
  |A|^2 = N / (s_{t s1} s_{s1 s2} ... s_{sm tb} s_{tb t}) with N independent of
  the ordering; so |A_sigma|^2 times the product of adjacent invariants is the
  same for every ordering.  Helicity configurations with fewer than two of
  either sign vanish.
* Lorentz invariance and Bose symmetry of the summed |M|^2 with five gluons.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import seeded_inputs as si

MT = 173.0
METRIC = np.array([1.0, -1.0, -1.0, -1.0])
G = oracle.gamma_matrices()


def slash(a):
    """gamma^mu a_mu for a (complex) contravariant four-vector a."""
    return np.einsum("m,mrc,m->rc", METRIC, G, np.asarray(a, dtype=complex))


def mdot(a, b):
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3]


def kinematics(ng, rs, seed, mt=MT):
    x = si.unit_points(64, si.ndim(ng), seed=seed)
    mom, wt = oracle.phase_space(ng, x, rs, mt)
    return mom[np.argmax(wt > 0)]


def helicities(m, h):
    """(gluon helicities, top, antitop) of the oracle's helicity index h."""
    lam = [1 if (h >> (m + 1 - i)) & 1 else -1 for i in range(m)]
    return lam, (1 if (h >> 1) & 1 else -1), (1 if h & 1 else -1)


def photon_amplitude(m, k_phys, incoming, pt, ptb, mt, h):
    """QED amplitude of the top line with m photons: sum over attachment orders of
    ubar(pt) eps1 S(q1) eps2 S(q2) ... eps_m v(ptb), S(q) = (qslash + m)/(q^2 - m^2),
    q_j = pt + (outgoing momenta of the first j photons), unit coupling."""
    lam, lt, ltb = helicities(m, h)
    eps, kout = [], []
    for i in range(m):
        if incoming[i]:
            eps.append(oracle.wavefunction("eps", k_phys[i], 0.0, lam[i]))
            kout.append(-np.asarray(k_phys[i], float))
        else:
            eps.append(oracle.wavefunction("eps*", k_phys[i], 0.0, lam[i]))
            kout.append(np.asarray(k_phys[i], float))
    ubar = oracle.wavefunction("ubar", pt, mt, lt)
    v = oracle.wavefunction("v", ptb, mt, ltb)
    total = 0.0 + 0.0j
    for order in itertools.permutations(range(m)):
        row = ubar @ slash(eps[order[0]])
        q = np.asarray(pt, float).copy()
        for j in range(1, m):
            q = q + kout[order[j - 1]]
            prop = (slash(q) + mt * np.eye(4)) / (mdot(q, q) - mt * mt)
            row = row @ prop @ slash(eps[order[j]])
        total += row @ v
    return total


@pytest.mark.parametrize("m,rs,seed", [(3, 1500.0, 61), (4, 2500.0, 62), (5, 3500.0, 63)])
def test_abelian_identity(m, rs, seed):
    mom = kinematics(m - 2, rs, seed)
    k = np.concatenate([mom[:2], mom[4:]])
    inc = [1, 1] + [0] * (m - 2)
    hs = range(1 << (m + 2)) if m < 5 else (0, 1, 6, 37, 77, 100, 127)
    sign = (-1) ** (m - 1)  # the recursion's fermion propagator carries -(pslash + m)/(p^2 - m^2)
    checked = 0
    for h in hs:
        A = oracle.partial_amplitudes(m, k, inc, mom[2], mom[3], MT, h)
        qed = photon_amplitude(m, k, inc, mom[2], mom[3], MT, h)
        scale = max(np.max(np.abs(A)), abs(qed))
        assert abs(A.sum() - sign * qed) <= 1e-11 * scale, (h, A.sum(), qed)
        # the identity is not trivially 0 = 0: the photon amplitude is sizeable
        checked += abs(qed) > 1e-3 * scale
    assert checked >= len(hs) // 2


def _adjacent_product(order, k_out, pt, ptb):
    """|s_{t s1}| |s_{s1 s2}| ... |s_{sm tb}| for the cyclic order t, s1..sm, tb (massless)."""
    chain = [pt] + [k_out[i] for i in order] + [ptb]
    out = 1.0
    for a, b in zip(chain[:-1], chain[1:]):
        out *= abs(2.0 * mdot(a, b))
    return out


@pytest.mark.parametrize("m,rs,seed", [(3, 1200.0, 71), (4, 1600.0, 72), (5, 2000.0, 73)])
def test_massless_parke_taylor_ratios(m, rs, seed):
    mom = kinematics(m - 2, rs, seed, mt=0.0)
    k = np.concatenate([mom[:2], mom[4:]])
    inc = [1, 1] + [0] * (m - 2)
    k_out = [(-k[i] if inc[i] else k[i]) for i in range(m)]
    perms = list(itertools.permutations(range(m)))
    D = np.array([_adjacent_product(p, k_out, mom[2], mom[3]) for p in perms])
    n_mhv = 0
    top = 0.0
    results = []
    for h in range(1 << (m + 2)):
        lam, lt, ltb = helicities(m, h)
        out_hel = [(-l if inc[i] else l) for i, l in enumerate(lam)] + [lt, ltb]
        neg = sum(1 for x in out_hel if x < 0)
        A = oracle.partial_amplitudes(m, k, inc, mom[2], mom[3], 0.0, h)
        top = max(top, np.max(np.abs(A)))
        results.append((neg, lt, ltb, A))
    n = m + 2
    for neg, lt, ltb, A in results:
        if lt == ltb or neg < 2 or neg > n - 2:
            # helicity conservation on the massless quark line, and the
            # all-but-one equal helicity amplitudes, vanish
            assert np.max(np.abs(A)) <= 1e-11 * top
        elif neg == 2 or neg == n - 2:
            n_mhv += 1
            r = np.abs(A) ** 2 * D
            assert np.max(np.abs(A)) > 1e-6 * top
            assert np.max(r) / np.min(r) - 1 < 1e-9, (neg, r.min(), r.max())
    # both quark helicity assignments times the m gluons carrying the second
    # negative (or second positive) helicity
    assert n_mhv == 2 * 2 * m if n > 4 else n_mhv == 2 * m


def test_lorentz_invariance_five_gluons():
    mom = kinematics(3, 3500.0, 45)
    L = si.boost_matrix(np.array([-0.2, 0.4, 0.35])) @ si.rotation_matrix(11)
    a = oracle.me_gg(5, mom, MT)
    b = oracle.me_gg(5, mom @ L.T, MT)
    assert abs(b / a - 1) < 1e-10


def test_bose_and_charge_conjugation_symmetry_five_gluons():
    mom = kinematics(3, 3500.0, 53)
    a = oracle.me_gg(5, mom, MT)
    for i, j in ((4, 5), (5, 6), (4, 6), (0, 1), (2, 3)):
        sw = mom.copy()
        sw[[i, j]] = sw[[j, i]]
        assert abs(oracle.me_gg(5, sw, MT) / a - 1) < 1e-11, (i, j)
