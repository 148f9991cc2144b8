"""CPU pin of the oracle's dynamic factorisation scale mu = H_T / 2: for each
event, the dynamic-scale weight equals the fixed-scale weight with mu set to
that event's H_T / 2, computed here from the event's momenta (half the sum
of the transverse masses of the two tops and the transverse momenta of the
gluons)."""
import numpy as np
import pytest

import oracle
import seeded_inputs as si

MT = 173.0


@pytest.mark.parametrize("ng", [0, 1, 2])
def test_dynamic_scale_is_half_ht_per_event(ng):
    d = si.ndim(ng)
    dr = 0.4 if ng >= 2 else 0.0
    dyn = oracle.Oracle(oracle.Config(n_g=ng, dr_min=dr, dyn_scale=True))
    x = si.points_above_threshold(40, d, 13000.0, MT, seed=60 + ng)
    w, mom = dyn.integrand_momenta(x)
    fixed = oracle.Oracle(oracle.Config(n_g=ng, dr_min=dr)).integrand(x)
    checked = 0
    for e in np.flatnonzero(w != 0.0)[:12]:
        t, tb, g = mom[e, 2], mom[e, 3], mom[e, 4:]
        ht = (np.sqrt(MT ** 2 + t[1] ** 2 + t[2] ** 2) + np.sqrt(MT ** 2 + tb[1] ** 2 + tb[2] ** 2)
              + np.sum(np.hypot(g[:, 1], g[:, 2])))
        ref = oracle.Oracle(oracle.Config(n_g=ng, dr_min=dr, mu=0.5 * ht)).integrand(x[e:e + 1])[0]
        assert abs(w[e] - ref) <= 1e-12 * abs(ref)
        checked += 1
    assert checked >= 8
    # the scale matters: the weights differ from the fixed-scale (mu = m_t) ones
    nz = w != 0.0
    assert np.max(np.abs(w[nz] / fixed[nz] - 1.0)) > 1e-3
