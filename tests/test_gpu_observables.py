"""Observable histograms of a VEGAS integration against the FP64 oracle.

The oracle side: the same Philox events through the same grid, the oracle's
weights and partonic centre-of-mass momenta, binned in numpy with the same
bin rule.  Both sides compute the observables and the bin decisions in FP64
from independent kinematics code; the per-bin sums agree to rounding
(1e-10 relative; an event within rounding of a bin edge would show up as a
single-event difference, which these seeds do not produce).
"""
import numpy as np
import pytest

import oracle
import seeded_inputs as si

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2105_10529_amd as mf  # noqa: E402

PROC = {0: "gg>ttx", 1: "gg>ttxg", 2: "gg>ttxgg"}
SPEC = {"nbins": 40, "lo": (0.0, 300.0, 0.0), "hi": (800.0, 2300.0, 600.0)}


def _oracle_hist(ng, edges, it, n, seed, spec):
    d = si.ndim(ng)
    orc = oracle.Oracle(oracle.Config(n_g=ng, dr_min=0.4 if ng >= 2 else 0.0))
    u = oracle.event_uniforms(n, d, it, seed, 0)
    xs = np.empty((n, d))
    jac = np.empty(n)
    for i in range(n):
        xs[i], jac[i], _ = oracle.vegas_map(edges, u[i])
    w, mom = orc.integrand_momenta(xs)
    w = w * jac
    top, atop = mom[:, 2], mom[:, 3]
    P = top + atop
    v = [np.hypot(top[:, 1], top[:, 2]),
         np.sqrt(np.maximum(P[:, 0] ** 2 - P[:, 1] ** 2 - P[:, 2] ** 2 - P[:, 3] ** 2, 0.0)),
         np.max(np.hypot(mom[:, 4:, 1], mom[:, 4:, 2]), axis=1) if ng > 0 else np.full(n, -1.0)]
    nb = spec["nbins"]
    out = np.zeros((3, nb, 2))
    for q in range(3):
        t = (v[q] - spec["lo"][q]) * (nb / (spec["hi"][q] - spec["lo"][q]))
        ok = (t >= 0.0) & (t < nb) & (w != 0.0)
        k = t[ok].astype(np.int64)
        np.add.at(out[q, :, 0], k, w[ok])
        np.add.at(out[q, :, 1], k, w[ok] ** 2)
    return out, w


@pytest.mark.parametrize("ng,precision,n,rtol", [(1, "fp64", 20000, 1e-10), (0, "fp64", 20000, 1e-10),
                                                 (2, "fp32", 3000, 1e-5)])
def test_histograms_match_oracle(ng, precision, n, rtol):
    d = si.ndim(ng)
    p = mf.Process(mf.Config(process=PROC[ng], precision=precision, dr_min=0.4 if ng >= 2 else 0.0))
    grid = si.random_grid(d, 50, seed=9)
    r = p.integrate(1, n, adapt=False, iter_offset=4, edges_in=torch.from_numpy(grid).to("cuda"),
                    observables=SPEC)
    got = r.observables["sums"]
    ref, w = _oracle_hist(ng, grid, 4, n, p.cfg.seed, SPEC)
    assert np.count_nonzero(ref[0, :, 0]) > 10
    scale = np.max(np.abs(ref), axis=1, keepdims=True)
    assert np.all(np.abs(got - ref) <= rtol * np.abs(ref) + 1e-14 * scale), np.max(np.abs(got - ref) / scale)
    if ng == 0:
        assert np.all(got[2] == 0.0)  # no final gluons
    # per-bin cross sections are the sums over N events
    assert np.allclose(r.observables["sigma_pb"], got[:, :, 0] / n)


def test_full_range_histogram_sums_to_the_integral():
    """With ranges covering every event, each observable's bins add up to the
    iteration's sum of weights (a property independent of the oracle)."""
    p = mf.Process(mf.Config(process="gg>ttxg"))
    p.integrate(3, 200_000, adapt=True)
    spec = {"nbins": 64, "lo": (0.0, 0.0, 0.0), "hi": (7000.0, 14000.0, 7000.0)}
    n = 2_000_000
    r = p.integrate(1, n, adapt=False, iter_offset=10, observables=spec)
    tot = r.observables["sums"][:, :, 0].sum(axis=1)
    assert np.allclose(tot / n, r.integral, rtol=1e-11, atol=0.0), (tot / n, r.integral)


def test_warmup_iterations_are_not_counted():
    ng, n = 1, 8000
    p = mf.Process(mf.Config(process=PROC[ng]))
    grid = si.random_grid(7, 50, seed=10)
    r = p.integrate(3, n, adapt=False, warmup=2, iter_offset=20, edges_in=torch.from_numpy(grid).to("cuda"),
                    observables=SPEC)
    ref, _ = _oracle_hist(ng, grid, 22, n, p.cfg.seed, SPEC)
    scale = np.max(np.abs(ref), axis=1, keepdims=True)
    assert np.all(np.abs(r.observables["sums"] - ref) <= 1e-10 * np.abs(ref) + 1e-14 * scale)
    assert r.observables["events"] == n


def test_unsupported_and_invalid_requests():
    p = mf.Process(mf.Config(process="gg>ttxg"))
    for bad in ({"nbins": 0, "lo": (0, 0, 0), "hi": (1, 1, 1)}, {"nbins": 65, "lo": (0, 0, 0), "hi": (1, 1, 1)},
                {"nbins": 8, "lo": (0, 5, 0), "hi": (1, 5, 1)}):
        with pytest.raises(mf.MFError) as e:
            p.integrate(1, 1000, observables=bad)
        assert e.value.status == mf.MF_EINVAL
    with pytest.raises(mf.MFError) as e:
        p.integrate(1, 1000, adapt=False, flow=mf.Flow(7, max_batch=1024), flow_mix=0.2, observables=SPEC)
    assert e.value.status == mf.MF_ENOTSUP
    g3 = mf.Process(mf.Config(process="gg>ttxggg", precision="fp32", dr_min=0.4))
    with pytest.raises(mf.MFError) as e:
        g3.integrate(1, 1000, observables=SPEC)
    assert e.value.status == mf.MF_ENOTSUP
