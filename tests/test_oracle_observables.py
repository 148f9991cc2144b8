"""CPU pins of the oracle's per-event momenta, which the observable
histograms of the GPU path are checked against: the momenta returned with
the weights belong to the same event (same weight as the plain integrand),
conserve four-momentum in the partonic centre-of-mass frame, put the tops on
their mass shell and the gluons on the light cone, and the full-range
histogram of any observable adds up to the VEGAS iteration's sum of weights.
"""
import numpy as np
import pytest

import oracle
import seeded_inputs as si

MT = 173.0


@pytest.mark.parametrize("ng", [0, 1, 2])
def test_momenta_belong_to_the_weighted_event(ng):
    d = si.ndim(ng)
    orc = oracle.Oracle(oracle.Config(n_g=ng, dr_min=0.4 if ng >= 2 else 0.0))
    x = si.points_above_threshold(200, d, 13000.0, MT, seed=40 + ng)
    w, mom = orc.integrand_momenta(x)
    assert np.array_equal(w, orc.integrand(x))
    # momenta are filled for events with kinematics (above the threshold of
    # the top pair after the gluon emissions); the others have zero weight
    has = mom[:, 0, 0] > 0.0
    assert np.all(w[~has] == 0.0) and np.count_nonzero(has) > 100
    w, mom = w[has], mom[has]
    E = mom[:, 0, 0]  # beam energy in the partonic frame
    p_in = mom[:, 0] + mom[:, 1]
    p_out = mom[:, 2:].sum(axis=1)
    assert np.max(np.abs(p_in - p_out) / E[:, None]) < 1e-12

    def m2(p):
        return p[..., 0] ** 2 - p[..., 1] ** 2 - p[..., 2] ** 2 - p[..., 3] ** 2

    for t in (2, 3):
        assert np.max(np.abs(m2(mom[:, t]) - MT ** 2) / E ** 2) < 1e-12
    if ng:
        assert np.max(np.abs(m2(mom[:, 4:])) / (E ** 2)[:, None]) < 1e-12


def test_full_range_histogram_is_the_iteration_sum():
    ng, n, d = 1, 400, 7
    orc = oracle.Oracle(oracle.Config(n_g=ng))
    grid = si.random_grid(d, 50, seed=11)
    S1, S2, _, _, _ = orc.vegas_iteration(grid, 3, n, 2105105290, purpose=0)
    u = oracle.event_uniforms(n, d, 3, 2105105290, 0)
    xs = np.empty((n, d))
    jac = np.empty(n)
    for i in range(n):
        xs[i], jac[i], _ = oracle.vegas_map(grid, u[i])
    w, mom = orc.integrand_momenta(xs)
    w = w * jac
    P = mom[:, 2] + mom[:, 3]
    mtt = np.sqrt(np.maximum(P[:, 0] ** 2 - (P[:, 1:] ** 2).sum(axis=1), 0.0))
    h, _ = np.histogram(mtt, bins=16, range=(0.0, 14000.0), weights=w)
    assert abs(h.sum() - S1) <= 1e-12 * abs(S1)
    assert abs(np.sum(w ** 2) - S2) <= 1e-12 * S2
