"""Build-time tables of the HIP path against the oracle (CPU).

The amplitude generator computes its colour matrices by colour-flow loop
counting; the oracle computes them from explicit Gell-Mann matrices.  The
tables of the g g -> t t~ g g g kernels (gluon order of each colour ordering,
gluon subsets of the contiguous ranges and suffixes) are checked against
their definition.
"""
import itertools
import os
import re
import sys

import numpy as np
import pytest

from oracle import colour

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_2105_10529_amd", "gen"))
import gen_me  # noqa: E402


@pytest.mark.parametrize("m", [2, 3, 4, 5])
def test_generator_colour_matrix_equals_oracle(m):
    perms, Z, den = gen_me.colour_matrix(m)
    assert perms == list(itertools.permutations(range(m)))
    C = np.array(Z, dtype=np.float64) / den
    assert np.allclose(C, colour.colour_matrix(m), rtol=0, atol=1e-9)


def _array(text, name):
    body = re.search(name + r"\[[^\]]*\](?:\[[^\]]*\])? = \{(.*?)\};", text, re.S).group(1)
    return [int(float(v)) for v in re.findall(r"-?\d+(?:\.\d+)?", body)]


def test_ttggg_pairs_differ_by_the_first_two_gluons():
    text = gen_me.emit_amp_tables(5)
    perms = list(itertools.permutations(range(5)))
    pairs = np.array(_array(text, "AMP_M5_PAIR")).reshape(-1, 2)
    assert len(pairs) == 60 and sorted(pairs.ravel().tolist()) == list(range(120))
    for a, b in pairs:
        pa, pb = perms[a], perms[b]
        assert pa[0] == pb[1] and pa[1] == pb[0] and pa[2:] == pb[2:]


def test_ttggg_tables_follow_their_definition():
    text = gen_me.emit_amp_tables(5)
    perms = list(itertools.permutations(range(5)))
    sig = np.array(_array(text, "AMP_M5_SIGMA")).reshape(120, 5)
    assert [tuple(r) for r in sig] == perms
    rng = np.array(_array(text, "AMP_M5_RANGE")).reshape(-1, 2)
    # every contiguous range of >= 2 positions once, by length then start
    want = [(a, a + ln - 1) for ln in range(2, 6) for a in range(0, 6 - ln)]
    assert [tuple(r) for r in rng] == want
    gm = np.array(_array(text, "AMP_M5_GMASK")).reshape(120, len(want))
    qm = np.array(_array(text, "AMP_M5_QMASK")).reshape(120, 4)
    for k, p in enumerate(perms):
        for r, (a, b) in enumerate(want):
            assert gm[k, r] == sum(1 << p[i] for i in range(a, b + 1))
        for j in range(4):
            assert qm[k, j] == sum(1 << p[i] for i in range(j + 1, 5))
    Z = np.array(_array(text, "AMP_M5_COLOUR"), dtype=np.float64).reshape(120, 120)
    den = float(re.search(r"AMP_M5_COLOUR_DEN = (\d+)", text).group(1))
    assert np.allclose(Z / den, colour.colour_matrix(5), rtol=0, atol=1e-9)
    # every numerator is an integer that FP32 holds exactly
    assert np.max(np.abs(Z)) < 2 ** 24


def test_flop_counts_are_consistent():
    fc = gen_me.amp_flop_count(5)
    assert fc["states"] == 64
    assert fc["colour_per_state"] == 2 * 2 * 2 * 120 * 120
    # per ordering: 10 gluon currents, 4 spinor currents, the closing sum and two contractions
    c = gen_me.COST
    per_ordering = (4 * (c["v3"] + c["vscale"]) + 3 * (2 * c["v3"] + c["w4"] + 2 * c["vadd"] + c["vscale"])
                    + 2 * (3 * c["v3"] + 3 * c["w4"] + 5 * c["vadd"] + c["vscale"])
                    + (4 * c["v3"] + 6 * c["w4"] + 9 * c["vadd"] + c["vscale"])
                    + sum(L * c["slash"] + (L - 1) * c["sadd"] + c["prop"] for L in range(1, 5))
                    + 5 * c["slash"] + 4 * c["sadd"] + 2 * c["ubar"])
    # a pair of orderings (first two gluons swapped) shares the currents of
    # positions 2..4: J(2,3), J(3,4), J(2,4) and the spinor currents from 4, 3, 2
    shared = (2 * (c["v3"] + c["vscale"]) + (2 * c["v3"] + c["w4"] + 2 * c["vadd"] + c["vscale"])
              + sum(L * c["slash"] + (L - 1) * c["sadd"] + c["prop"] for L in range(1, 4)))
    assert shared == 715
    assert fc["amplitudes_single_state"] == 120 * per_ordering - 60 * shared
    # the summed mode builds the gluon currents once for both antitop helicities
    gluon = (4 * (c["v3"] + c["vscale"]) + 3 * (2 * c["v3"] + c["w4"] + 2 * c["vadd"] + c["vscale"])
             + 2 * (3 * c["v3"] + 3 * c["w4"] + 5 * c["vadd"] + c["vscale"])
             + (4 * c["v3"] + 6 * c["w4"] + 9 * c["vadd"] + c["vscale"]))
    gluon_shared = 2 * (c["v3"] + c["vscale"]) + (2 * c["v3"] + c["w4"] + 2 * c["vadd"] + c["vscale"])
    assert fc["gluon_currents_per_state"] == 120 * gluon - 60 * gluon_shared
    assert fc["amplitudes_per_state"] == fc["amplitudes_single_state"] - fc["gluon_currents_per_state"] // 2
    assert fc["total"] == 64 * (fc["amplitudes_per_state"] + fc["colour_per_state"])



def test_shared_antitop_counts():
    """g g -> t t~ g and g g -> t t~ g g build each ordering's gluon currents
    once per gluon polarisation state for both antitop helicities: the count
    drops by one set of gluon currents per gluon polarisation state."""
    for m, before in ((3, 51882), (4, 680186)):
        fc = gen_me.flop_count(m)
        assert fc["total"] == before - (fc["states"] // 2) * fc["gluon_currents_per_polarisation"]


def test_two_line_colour_matrix_matches_oracle():
    """The generator's colour matrix of the quark channels (Fierz loop
    counting over products of traces) equals the oracle's explicit Gell-Mann
    sum."""
    from oracle import colour

    CC = gen_me.two_line_colour_matrix()
    got = np.array([[float(re_) + 1j * float(im_) for re_, im_ in row] for row in CC])
    assert np.allclose(got, colour.two_line_colour_matrix(), atol=1e-13)


def test_multi_trace_sum_small_cases():
    from fractions import Fraction

    assert gen_me.multi_trace_sum([()]) == 3  # Tr(1) = N
    assert gen_me.multi_trace_sum([(0,), (0,)]) == 0  # Tr(t^a) = 0
    assert gen_me.multi_trace_sum([(0, 1), (0, 1)]) == 2  # Tr(t^a t^b)^2 = (N^2 - 1)/4
    assert gen_me.multi_trace_sum([(0, 1, 0, 1)]) == gen_me.trace_sum((0, 1, 0, 1)) == Fraction(-2, 3)
