"""Dynamic factorisation scale mu = H_T / 2 on the GPU against the FP64 oracle
with the same scale (whose per-event scale is pinned on the CPU): the full
(x, Q) PDF interpolation per event.  Tolerances as for the fixed scale:
1e-11 per event in FP64, 1e-5 with FP32 amplitudes."""
import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import assert_close, to_dev_soa

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2105_10529_amd as mf  # noqa: E402

SQRT_S, MT = 13000.0, 173.0
PROC = {0: "gg>ttx", 1: "gg>ttxg", 2: "gg>ttxgg", 3: "gg>ttxggg"}


def _pair(ng, precision="fp64", channel="gg", process=None):
    dr = 0.4 if ng >= 2 else 0.0
    p = mf.Process(mf.Config(process=process or PROC[ng], precision=precision, dr_min=dr, dynamic_scale=True))
    o = oracle.Oracle(oracle.Config(n_g=ng, channel=channel, dr_min=dr, dyn_scale=True))
    return p, o


@pytest.mark.parametrize("ng,precision,n,rtol", [(0, "fp64", 3000, 1e-11), (1, "fp64", 3000, 1e-11),
                                                 (2, "fp64", 400, 1e-11), (2, "fp32", 400, 1e-5),
                                                 (3, "fp32", 120, 1e-5)])
def test_integrand_matches_oracle(ng, precision, n, rtol):
    p, o = _pair(ng, precision)
    d = si.ndim(ng)
    x = np.concatenate([si.points_above_threshold(n, d, SQRT_S, MT, seed=70 + ng), si.edge_points(d)])
    ref = o.integrand(x)
    got = p.integrand(to_dev_soa(x)).cpu().numpy()
    assert np.count_nonzero(ref) > n // 3
    assert_close(got, ref, rtol)
    # the scale is not the fixed one
    fixed = mf.Process(mf.Config(process=PROC[ng], precision=precision,
                                 dr_min=0.4 if ng >= 2 else 0.0)).integrand(to_dev_soa(x)).cpu().numpy()
    nz = ref != 0.0
    assert np.max(np.abs(fixed[nz] / got[nz] - 1.0)) > 1e-3


def test_quark_channel_matches_oracle():
    p, o = _pair(0, channel="uu~", process="uux>ttx")
    x = si.points_above_threshold(2000, 4, SQRT_S, MT, seed=75)
    assert_close(p.integrand(to_dev_soa(x)).cpu().numpy(), o.integrand(x), 1e-11)


def test_vegas_iteration_matches_oracle():
    p, o = _pair(1)
    grid = si.random_grid(7, 50, seed=12)
    r = p.integrate(1, 20000, adapt=False, iter_offset=7, edges_in=torch.from_numpy(grid).to("cuda"))
    S1, S2, _, nnz, nbad = o.vegas_iteration(grid, 7, 20000, p.cfg.seed, purpose=0)
    I, s = oracle.iteration_estimate(S1, S2, 20000)
    assert abs(r.iter_integral[0] / I - 1) < 1e-12
    assert r.n_nonzero == nnz and nbad == 0


def test_derivatives_and_invalid_values_are_refused():
    p, _ = _pair(1)
    x = to_dev_soa(si.points_above_threshold(8, 7, SQRT_S, MT, seed=76))
    with pytest.raises(mf.MFError) as e:
        p.integrand_grad(x)
    assert e.value.status == mf.MF_ENOTSUP
    with pytest.raises(mf.MFError) as e:
        p.grad(100_000)
    assert e.value.status == mf.MF_ENOTSUP
    cfg = mf.Config(process="gg>ttxg")
    cfg.dynamic_scale = 2
    with pytest.raises(mf.MFError) as e:
        mf.Process(cfg)
    assert e.value.status == mf.MF_EINVAL
