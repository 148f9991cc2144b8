"""HIP path vs the FP64 oracle, element by element on identical seeded inputs.

Tolerances: FP64 amplitudes agree with the oracle to 1e-11 relative per event
(two independent FP64 evaluations of the same definition, which differ only
in rounding order; cancellations between colour orderings cost a few digits
at most).  FP32 amplitudes: |dME|/ME <= 1e-5 per event is the target of the
FP32 mode; the test bound is the same.
"""
import math

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from gpu_util import assert_close, rel_err, to_dev_soa

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

import paper_2105_10529_amd as mf  # noqa: E402

SQRT_S, MT = 13000.0, 173.0
PROC = {0: "gg>ttx", 1: "gg>ttxg", 2: "gg>ttxgg"}


def _oracle(ng, channel="gg", dr=None):
    return oracle.Oracle(oracle.Config(n_g=ng, channel=channel, dr_min=(0.4 if ng >= 2 else 0.0) if dr is None else dr))


def _proc(ng, precision="fp64", process=None, dr=None, colour_form=0):
    return mf.Process(mf.Config(process=process or PROC[ng], precision=precision,
                                dr_min=(0.4 if ng >= 2 else 0.0) if dr is None else dr, colour_form=colour_form))


def _points(n, d, seed):
    x = si.points_above_threshold(n, d, SQRT_S, MT, seed=seed)
    return np.concatenate([x, si.edge_points(d)])


@pytest.mark.parametrize("ng,n", [(0, 4099), (1, 3001), (2, 600)])
def test_integrand_fp64_matches_oracle(ng, n):
    d = si.ndim(ng)
    x = _points(n, d, 100 + ng)
    ref = _oracle(ng).integrand(x)
    got = _proc(ng).integrand(to_dev_soa(x)).cpu().numpy()
    assert np.count_nonzero(ref) > 0.5 * n
    assert_close(got, ref, 1e-11)


@pytest.mark.parametrize("channel,process", [("uu~", "uux>ttx"), ("dd~", "ddx>ttx")])
def test_quark_channels_match_oracle(channel, process):
    x = _points(2000, 4, 7)
    ref = _oracle(0, channel).integrand(x)
    got = _proc(0, process=process).integrand(to_dev_soa(x)).cpu().numpy()
    assert_close(got, ref, 1e-11)


@pytest.mark.parametrize("ng,n", [(0, 2000), (1, 2000), (2, 500)])
def test_integrand_fp32_amplitudes_within_1e5(ng, n):
    d = si.ndim(ng)
    x = _points(n, d, 200 + ng)
    ref = _oracle(ng).integrand(x)
    got = _proc(ng, "fp32").integrand(to_dev_soa(x)).cpu().numpy()
    e = rel_err(got, ref, floor=1e-20 * np.max(np.abs(ref)))
    print(f"fp32 |dw|/w: median {np.median(e):.2e} q999 {np.quantile(e, 0.999):.2e} max {np.max(e):.2e}")
    assert_close(got, ref, 1e-5)


def test_empty_ragged_and_single_inputs():
    p = _proc(1)
    u = torch.empty((7, 0), dtype=torch.float64, device="cuda")
    assert p.integrand(u).numel() == 0
    orc = _oracle(1)
    for n in (1, 63, 65, 257):
        x = _points(n, 7, 300 + n)[:n]
        got = p.integrand(to_dev_soa(x)).cpu().numpy()
        assert_close(got, orc.integrand(x), 1e-11)


def test_invalid_configurations_raise():
    with pytest.raises(mf.MFError) as e:
        mf.Process(mf.Config(sqrt_s=300.0))
    assert e.value.status == mf.MF_EINVAL
    with pytest.raises(mf.MFError) as e:
        mf.Process(mf.Config(n_bins=0))
    assert e.value.status == mf.MF_EINVAL
    with pytest.raises(mf.MFError) as e:
        mf.Process(mf.Config(mu=1e6))
    assert e.value.status == mf.MF_ERANGE


@pytest.mark.parametrize("ng,n,precision", [(0, 20000, "fp64"), (1, 20000, "fp64"), (2, 3000, "fp64"),
                                            (1, 20000, "fp32"), (2, 3000, "fp32")])
def test_vegas_iteration_matches_oracle_exactly(ng, n, precision):
    """One on-device iteration (same Philox stream) against the oracle's loop.

    FP64: equal to rounding (1e-12 on the iteration estimate); FP32 amplitudes:
    every weight within 1e-5 of the FP64 oracle, so the mean is within 1e-5.
    """
    tol = 1e-12 if precision == "fp64" else 1e-5
    p = _proc(ng, precision)
    orc = _oracle(ng)
    d = si.ndim(ng)
    edges = torch.from_numpy(si.random_grid(d, 50, seed=5)).to("cuda")
    out = torch.empty_like(edges)
    r = p.integrate(1, n, adapt=True, iter_offset=3, edges_in=edges, edges_out=out)
    S1, S2, hist, nnz, nbad = orc.vegas_iteration(si.random_grid(d, 50, seed=5), 3, n, p.cfg.seed, purpose=0)
    I, s = oracle.iteration_estimate(S1, S2, n)
    assert abs(r.iter_integral[0] / I - 1) < tol
    assert abs(r.iter_error[0] / s - 1) < (1e-9 if precision == "fp64" else 1e-4)
    assert r.n_nonzero == nnz and r.n_nonfinite == nbad == 0
    ref_edges = oracle.vegas_refine(si.random_grid(d, 50, seed=5), hist, 1.5)
    assert np.max(np.abs(out.cpu().numpy() - ref_edges)) < (1e-10 if precision == "fp64" else 1e-5)


_FULL_GEOMETRY_ORACLE = {}


def _oracle_iteration(ng, n, grid_seed, iteration, seed):
    key = (ng, n, grid_seed, iteration, seed)
    if key not in _FULL_GEOMETRY_ORACLE:
        d = si.ndim(ng)
        _FULL_GEOMETRY_ORACLE[key] = _oracle(ng).vegas_iteration(si.random_grid(d, 50, seed=grid_seed), iteration, n,
                                                                 seed, purpose=0)
    return _FULL_GEOMETRY_ORACLE[key]


@pytest.mark.parametrize("ng,n,precision,form", [(1, 1_100_000, "fp64", 0), (2, 600_000, "fp32", 1),
                                                 (2, 600_000, "fp32", 2), (2, 600_000, "fp64", 1),
                                                 (2, 600_000, "fp64", 2)])
def test_vegas_iteration_full_geometry_matches_oracle(ng, n, precision, form):
    """One iteration in the looping geometry of the full-size runs: blocks of
    256 threads, each looping over several 256-event chunks (an iteration has
    at least 16 chunks per block once it has more than 256 chunks: 600000
    events run on 256 blocks of 9 or 10 chunks, 1100000 on 512 blocks of 8 or
    9, the last pass ragged).  That carried path -- per-wave LDS accumulators and
    histograms and the per-block lists of kept events persisting across
    chunks -- must give the oracle's iteration: FP64 to rounding (1e-12 on the
    estimate, 1e-10 on the refined edges, the same count of non-zero events),
    FP32 amplitudes within 1e-5.  g g -> t t~ g g with the colour form in
    registers (form 1; a fused kernel in FP32, a staged iteration -- points,
    integrand, accumulation -- in FP64) and on the matrix cores (form 2;
    staged, the integrand as selection, amplitude and colour kernels over
    chunks of at most 65536 passing events, so ~2.5 chunks here)."""
    fp64 = precision == "fp64"
    p = _proc(ng, precision, colour_form=form)
    d = si.ndim(ng)
    print(f"full geometry ng={ng} n={n} {precision} colour form {form}", flush=True)
    edges = torch.from_numpy(si.random_grid(d, 50, seed=15)).to("cuda")
    out = torch.empty_like(edges)
    r = p.integrate(1, n, adapt=True, iter_offset=5, edges_in=edges, edges_out=out)
    S1, S2, hist, nnz, nbad = _oracle_iteration(ng, n, 15, 5, p.cfg.seed)
    I, s = oracle.iteration_estimate(S1, S2, n)
    assert abs(r.iter_integral[0] / I - 1) < (1e-12 if fp64 else 1e-5), (r.iter_integral[0], I)
    assert abs(r.iter_error[0] / s - 1) < (1e-9 if fp64 else 1e-4)
    assert r.n_nonzero == nnz and r.n_nonfinite == nbad == 0
    ref_edges = oracle.vegas_refine(si.random_grid(d, 50, seed=15), hist, 1.5)
    assert np.max(np.abs(out.cpu().numpy() - ref_edges)) < (1e-10 if fp64 else 1e-5)


_TTGG_POINTS = {}


def _ttgg_points_and_oracle(n):
    if n not in _TTGG_POINTS:
        x = _points(n, 10, 210)
        _TTGG_POINTS[n] = (x, _oracle(2).integrand(x))
    return _TTGG_POINTS[n]


@pytest.mark.parametrize("precision,form", [("fp64", 1), ("fp64", 2), ("fp32", 1), ("fp32", 2)])
def test_gg_ttgg_colour_forms_match_oracle(precision, form):
    """g g -> t t~ g g per event against the FP64 oracle with the colour form
    in registers (1) and on the matrix cores (2; products of the exact
    integer numerators of the colour matrix, FP32 or FP64 accumulation), on
    140000 points (about 70000 pass the cuts: two chunks of the matrix-core
    path, the second ragged) plus the extreme uniforms."""
    x, ref = _ttgg_points_and_oracle(140_000)
    print(f"ttgg colour form {form} {precision}", flush=True)
    got = _proc(2, precision, colour_form=form).integrand(to_dev_soa(x)).cpu().numpy()
    assert np.count_nonzero(ref) > 65536
    assert_close(got, ref, 1e-11 if precision == "fp64" else 1e-5)


def test_gg_ttgg_fp64_colour_forms_agree():
    """The two FP64 colour forms sum the same exact quadratic form in a
    different order: per event they agree to rounding."""
    x = _points(3000, 10, 211)
    u = to_dev_soa(x)
    a = _proc(2, "fp64", colour_form=1).integrand(u).cpu().numpy()
    b = _proc(2, "fp64", colour_form=2).integrand(u).cpu().numpy()
    assert_close(b, a, 1e-13)
    with pytest.raises(mf.MFError) as e:
        _proc(1, colour_form=2)
    assert e.value.status == mf.MF_ENOTSUP
    with pytest.raises(mf.MFError) as e:
        _proc(2, colour_form=3)
    assert e.value.status == mf.MF_EINVAL


def test_refine_matches_oracle():
    d, nb = 7, 50
    rng = np.random.default_rng(9)
    for trial in range(4):
        e = si.random_grid(d, nb, seed=trial)
        h = rng.exponential(size=(d, nb)) ** 3
        h[1, :] = 0.0  # an all-zero dimension is left unchanged
        h[2, 10:20] = 0.0
        ed = torch.from_numpy(e).to("cuda")
        mf.vegas_refine(ed, torch.from_numpy(h).to("cuda"))
        ref = oracle.vegas_refine(e, h)
        assert np.max(np.abs(ed.cpu().numpy() - ref)) < 1e-12
        assert np.array_equal(ed.cpu().numpy()[1], e[1])


def test_gg_ttbar_cross_section_matches_quadrature():
    from oracle import quad

    ref = quad.hadronic_sigma(_oracle(0), "gg")
    r = _proc(0).integrate(5, 100000)
    assert abs(r.integral - ref) < 3 * r.error
    assert r.error / r.integral < 5e-3


def test_quark_cross_section_matches_quadrature():
    from oracle import quad

    ref = quad.hadronic_sigma(_oracle(0, "uu~"), "qq")
    ru = _proc(0, process="uux>ttx").integrate(5, 100000)
    rd = _proc(0, process="ddx>ttx").integrate(5, 100000)
    assert abs(ru.integral + rd.integral - ref) < 3 * math.hypot(ru.error, rd.error)


def test_full_size_iteration_is_deterministic_and_consistent():
    """gg -> t t~ g at 1e7 events per iteration (the benchmark's launch shape):
    bitwise reproducible, and statistically consistent with the oracle's own
    estimate on an independent stream."""
    p = _proc(1)
    d = 7
    edges = torch.from_numpy(si.random_grid(d, 50, seed=11)).to("cuda")
    a = p.integrate(1, 10_000_000, adapt=False, edges_in=edges)
    b = p.integrate(1, 10_000_000, adapt=False, edges_in=edges)
    assert a.iter_integral[0] == b.iter_integral[0] and a.iter_error[0] == b.iter_error[0]
    orc = _oracle(1)
    S1, S2, _, _, _ = orc.vegas_iteration(si.random_grid(d, 50, seed=11), 0, 200000, 12345, purpose=2)
    I, s = oracle.iteration_estimate(S1, S2, 200000)
    assert abs(a.iter_integral[0] - I) < 4 * math.hypot(a.iter_error[0], s)


@pytest.mark.parametrize("ng,precision", [(0, "fp64"), (1, "fp64"), (1, "fp32")])
def test_gradients_match_oracle(ng, precision):
    d = si.ndim(ng)
    x = _points(400, d, 400 + ng)
    orc = _oracle(ng)
    p = _proc(ng, precision)
    w, dw = p.integrand_grad(to_dev_soa(x))
    w, dw = w.cpu().numpy(), dw.cpu().numpy()
    tol = 1e-10 if precision == "fp64" else 2e-5
    for k, direction in enumerate(range(1, 10)):
        rw, rdw = orc.integrand_grad(x, direction)
        if k == 0:
            assert_close(w, rw, 1e-11 if precision == "fp64" else 1e-5)
        scale = max(np.max(np.abs(rdw)), 1e-300)
        assert np.max(np.abs(dw[k] - rdw)) < tol * scale, k


def test_grad_estimator_matches_oracle_sum():
    """mf_grad over Philox events equals the oracle's mean over the same events."""
    p = _proc(1)
    d = 7
    n = 4000
    vals, errs = p.grad(n, iter_offset=2)
    orc = _oracle(1)
    u = oracle.event_uniforms(n, d, 2, p.cfg.seed, 0)
    # uniform grid: x = u, Jacobian 1
    w, _ = orc.integrand_grad(u, 2)
    assert abs(vals[0] / w.mean() - 1) < 1e-12
    for k, direction in enumerate(range(1, 10)):
        _, dw = orc.integrand_grad(u, direction)
        ref = dw.mean()
        assert abs(vals[1 + k] - ref) <= 1e-10 * max(abs(ref), np.abs(dw).max() / n), k


def test_mt_derivative_per_event_matches_central_differences():
    """Per event, at explicit points: d w / d m_t from the forward-mode kernel
    against (w(m_t + h) - w(m_t - h)) / 2h with h = 0.05 GeV, both in FP64.
    The gluon momenta and the cuts do not depend on m_t (the gluons are
    emitted before the top pair is split), so each event's weight is a
    smooth function of m_t except through the top-pair threshold, where
    w ~ beta = sqrt(1 - 4 m_t^2 / M_tt^2) has no Taylor expansion; events
    with M_tt > 2 (m_t + 10 GeV) (those still above threshold at
    m_t + 10 GeV) have a central-difference error of order (h / 20 GeV)^2
    < 1e-5, checked at 1e-4."""
    d = 7
    x = _points(20000, d, 55)
    u = to_dev_soa(x)
    h = 0.05
    w0, dw = _proc(1).integrand_grad(u)
    dw = dw[0].cpu().numpy()
    wp = mf.Process(mf.Config(process="gg>ttxg", m_t=MT + h)).integrand(u).cpu().numpy()
    wm = mf.Process(mf.Config(process="gg>ttxg", m_t=MT - h)).integrand(u).cpu().numpy()
    far = mf.Process(mf.Config(process="gg>ttxg", m_t=MT + 10.0)).integrand(u).cpu().numpy() != 0.0
    fd = (wp - wm) / (2 * h)
    assert far.sum() > 5000
    err = np.abs(fd[far] - dw[far])
    assert np.all(err <= 1e-4 * np.abs(dw[far]) + 1e-10 * np.abs(dw[far]).max()), float(
        np.max(err / np.abs(dw[far])))


def test_derivatives_match_central_differences_on_the_same_events():
    """dsigma/dm_t and dsigma/dtheta from the pathwise estimator against
    central differences of sigma computed from the same Philox events on the
    same frozen grid: h = 0.05 GeV for m_t, relative 1e-4 for the PDF
    parameters (their derivative is exact in the kinematics, so only O(h^2)
    remains, checked at 1e-6).  For m_t the cuts cannot move (they act on
    the gluons, whose momenta do not depend on m_t) and the threshold adds no
    boundary term (the weight vanishes there like beta); the two estimates
    differ only through the events within a few h of the top-pair threshold,
    where w ~ beta has no Taylor expansion and the central difference of
    each such event differs from its derivative by O(1) (the per-event test
    above covers the events away from it).  Their share of the estimate is of
    order sqrt(h / m_t) times the fraction of the cross section near
    threshold; the bound is 1e-3."""
    p = _proc(1)
    p.integrate(3, 200_000, adapt=True)
    edges = torch.empty((7, 51), dtype=torch.float64, device="cuda")
    p.integrate(1, 2, adapt=False, edges_out=edges, iter_offset=99)
    n = 1_000_000
    vals, errs = p.grad(n, iter_offset=7, edges_in=edges)

    def sigma(**kw):
        q = mf.Process(mf.Config(process="gg>ttxg", **kw))
        return q.grad(n, iter_offset=7, edges_in=edges)[0][0]

    h = 0.05
    fd = (sigma(m_t=MT + h) - sigma(m_t=MT - h)) / (2 * h)
    assert abs(fd - vals[1]) < 1e-3 * abs(vals[1]), (fd, vals[1], errs[1])
    print(f"d sigma / d m_t: pathwise {vals[1]:.8g}, central difference {fd:.8g}, "
          f"relative difference {abs(fd / vals[1] - 1):.2e}")
    base = list(mf.DEFAULT_PDF)
    # out[2 + t] is d sigma / d theta_t; theta_1..4 = a_g, b_g, c_g, d_g = pdf_params[1..4]
    for k, idx in ((3, 1), (4, 2), (5, 3), (6, 4)):
        hp = 1e-4 * abs(base[idx])
        up, dn = list(base), list(base)
        up[idx] += hp
        dn[idx] -= hp
        fd = (sigma(pdf_params=tuple(up)) - sigma(pdf_params=tuple(dn))) / (2 * hp)
        assert abs(fd - vals[k]) < 1e-6 * abs(vals[k]), (idx, fd, vals[k])


def test_autograd_function_routes_the_kernel_derivatives():
    """torch.autograd over mf_integrand_grad: gradients of mean(w) with respect
    to m_t and theta equal the oracle's mean derivatives at the same points."""
    d = 7
    x = _points(500, d, 77)
    p = _proc(1)
    F = mf.make_autograd_integrand(p)
    mt = torch.tensor(MT, dtype=torch.float64, requires_grad=True)
    th = torch.tensor([p.cfg.pdf_params[i] for i in (0, 1, 2, 3, 4, 5, 10, 15)], dtype=torch.float64,
                      requires_grad=True)
    w = F.apply(to_dev_soa(x), mt, th)
    w.mean().backward()
    orc = _oracle(1)
    for k, direction in enumerate(range(1, 10)):
        _, rdw = orc.integrand_grad(x, direction)
        got = mt.grad.item() if k == 0 else th.grad[k - 1].item()
        assert abs(got - rdw.mean()) <= 1e-10 * max(abs(rdw.mean()), np.abs(rdw).max() / x.shape[0]), k
    with pytest.raises(ValueError):
        F.apply(to_dev_soa(x), torch.tensor(MT + 1.0, dtype=torch.float64), th)


def test_fp32_subsample_of_an_adapted_iteration_matches_the_oracle():
    """The Philox events of one iteration on an adapted g g -> t t~ g g grid:
    FP32-amplitude weights within 1e-5 of the FP64 oracle per event (same
    events, same grid, same cut decisions) and FP64 weights within 1e-10:
    the subsample of an adapted grid can hold events whose PDF value sits
    close to the interpolant's zero crossing near x -> 1, where the two
    sides' different interpolation orders (the GPU collapses Q first, the
    oracle interpolates x first) round differently relative to the small
    value (up to 7.4e-11 observed on 1e5 events); the element-by-element
    tests on random points keep 1e-11."""
    import bench

    r = bench.fp32_subsample_check(4000)
    assert r["same_zero_pattern"] and r["nonzero"] > 1000, r
    assert r["fp32_per_event_rel_err_max"] <= 1e-5, r
    assert r["fp64_per_event_rel_err_max"] <= 1e-10, r
    assert r["fp32_integral_rel_err"] <= 1e-6, r


def test_vjp_is_the_ordered_contraction():
    rng = np.random.default_rng(91)
    for k, n in ((9, 1), (9, 1000), (3, 300001)):
        dw = rng.normal(size=(k, n))
        g = rng.normal(size=n)
        got = mf.vjp(torch.from_numpy(dw).cuda(), torch.from_numpy(g).cuda()).cpu().numpy()
        ref = dw @ g
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(dw).sum(axis=1).max())


def test_handle_free_calls_work_in_caller_scratch():
    """mf_vjp, mf_weight_stats and mf_vegas_refine allocate nothing: they run
    in the scratch the caller passes, refuse a workspace smaller than the
    size they report (or misaligned) with MF_EINVAL before touching the
    device, and give the same bits with a reused, dirty workspace."""
    import ctypes

    L = mf.lib()
    rng = np.random.default_rng(93)
    k, n = 9, 70001
    dw = torch.from_numpy(rng.normal(size=(k, n))).cuda()
    g = torch.from_numpy(rng.normal(size=n)).cuda()
    need = L.mf_vjp_workspace(k, n)
    assert need >= 8 * k and L.mf_vjp_workspace(0, n) == 0
    out = torch.empty(k, dtype=torch.float64, device="cuda")
    work = torch.full(((need + 7) // 8 + 1,), float("nan"), dtype=torch.float64, device="cuda")
    assert L.mf_vjp(dw.data_ptr(), k, g.data_ptr(), n, out.data_ptr(), work.data_ptr(), need - 8, None) == mf.MF_EINVAL
    assert L.mf_vjp(dw.data_ptr(), k, g.data_ptr(), n, out.data_ptr(), work.data_ptr() + 4, need, None) == mf.MF_EINVAL
    assert L.mf_vjp(dw.data_ptr(), k, g.data_ptr(), n, out.data_ptr(), None, need, None) == mf.MF_EINVAL
    assert L.mf_vjp(dw.data_ptr(), k, g.data_ptr(), n, out.data_ptr(), work.data_ptr(), need, None) == mf.MF_OK
    first = out.cpu().numpy().copy()
    assert L.mf_vjp(dw.data_ptr(), k, g.data_ptr(), n, out.data_ptr(), work.data_ptr(), need, None) == mf.MF_OK
    assert np.array_equal(out.cpu().numpy(), first)
    assert np.array_equal(first, mf.vjp(dw, g).cpu().numpy())

    w = torch.from_numpy(np.abs(rng.normal(size=n))).cuda()
    need = L.mf_weight_stats_workspace(n)
    res = np.zeros(5)
    work = torch.full(((need + 7) // 8,), float("nan"), dtype=torch.float64, device="cuda")
    assert L.mf_weight_stats(w.data_ptr(), n, 0.5, res.ctypes.data, work.data_ptr(), need - 8, None) == mf.MF_EINVAL
    assert L.mf_weight_stats(w.data_ptr(), n, 0.5, res.ctypes.data, work.data_ptr(), need, None) == mf.MF_OK
    ref = mf.weight_stats(w, 0.5)
    assert res[0] == ref["mean"] and res[1] == ref["max"] and res[2] == ref["quantile"]
    assert res[2] == np.sort(w.cpu().numpy())[int(np.ceil(0.5 * n)) - 1]

    e = torch.from_numpy(si.random_grid(3, 50, seed=94)).cuda()
    h = torch.from_numpy(rng.random((3, 50)) + 0.1).cuda()
    st = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    assert L.mf_vegas_refine(e.data_ptr(), h.data_ptr(), 3, 50, 1.5, None, None) == mf.MF_EINVAL
    e2 = e.clone()
    assert L.mf_vegas_refine(e2.data_ptr(), h.data_ptr(), 3, 50, 1.5, st.data_ptr(), None) == mf.MF_OK
    assert int(st.item()) == 0
    assert np.max(np.abs(e2.cpu().numpy() - oracle.vegas_refine(si.random_grid(3, 50, seed=94), h.cpu().numpy()))) < 1e-10


QUARK_PROCS = [("uux>ttxg", "uu~"), ("ddx>ttxg", "dd~"), ("qg>ttxq", "qg")]


@pytest.mark.parametrize("process,channel", QUARK_PROCS)
def test_quark_channels_with_a_jet_match_oracle(process, channel):
    """u u~ -> t t~ g, d d~ -> t t~ g and q g -> t t~ q (+ q~ g) per event
    against the FP64 oracle's five-diagram evaluation (1e-11), points above
    threshold plus the extreme uniforms."""
    x = _points(3000, 7, 230)
    ref = oracle.Oracle(oracle.Config(n_g=1, channel=channel)).integrand(x)
    print(f"quark channel {process}", flush=True)
    got = mf.Process(mf.Config(process=process)).integrand(to_dev_soa(x)).cpu().numpy()
    assert np.count_nonzero(ref) > 1000
    assert_close(got, ref, 1e-11)


@pytest.mark.parametrize("process,channel", QUARK_PROCS)
def test_quark_channel_iteration_and_derivatives_match_oracle(process, channel):
    """One on-device VEGAS iteration equals the oracle's on the same Philox
    stream (1e-12), and the forward-mode derivatives in m_t and the eight PDF
    parameters equal the oracle's dual numbers per event (1e-10 of the largest
    value); the quark normalisations A_u, A_d, A_u~ now enter (non-zero
    derivatives), and d w / d A_f = w_f / A_f for the part of w with that
    flavour."""
    p = mf.Process(mf.Config(process=process))
    orc = oracle.Oracle(oracle.Config(n_g=1, channel=channel))
    edges = torch.from_numpy(si.random_grid(7, 50, seed=25)).to("cuda")
    out = torch.empty_like(edges)
    n = 20000
    r = p.integrate(1, n, adapt=True, iter_offset=4, edges_in=edges, edges_out=out)
    S1, S2, hist, nnz, _ = orc.vegas_iteration(si.random_grid(7, 50, seed=25), 4, n, p.cfg.seed, purpose=0)
    I, s = oracle.iteration_estimate(S1, S2, n)
    assert abs(r.iter_integral[0] / I - 1) < 1e-12 and r.n_nonzero == nnz
    assert np.max(np.abs(out.cpu().numpy() - oracle.vegas_refine(si.random_grid(7, 50, seed=25), hist))) < 1e-10
    x = _points(400, 7, 231)
    w, dw = p.integrand_grad(to_dev_soa(x))
    w, dw = w.cpu().numpy(), dw.cpu().numpy()
    for k, direction in enumerate(range(1, 10)):
        rw, rdw = orc.integrand_grad(x, direction)
        if k == 0:
            assert_close(w, rw, 1e-11)
        scale = max(np.max(np.abs(rdw)), 1e-300)
        assert np.max(np.abs(dw[k] - rdw)) < 1e-10 * scale, (process, k)
    # the quark normalisations the channel uses have non-zero derivatives
    used = {"uux>ttxg": (6, 8), "ddx>ttxg": (7, 8), "qg>ttxq": (6, 7, 8)}[process]
    for k in used:
        assert np.count_nonzero(dw[k]) > 100, (process, k)
    for k in set((6, 7, 8)) - set(used):
        assert np.all(dw[k] == 0.0), (process, k)


def test_quark_channel_derivative_matches_central_difference():
    """d sigma / d A_u of q g -> t t~ q from the pathwise estimator against a
    central difference of sigma on the same Philox events (h = 1e-4 A_u):
    sigma is linear in A_u, so they agree to rounding (1e-8)."""
    p = mf.Process(mf.Config(process="qg>ttxq"))
    n = 200_000
    vals, _ = p.grad(n, iter_offset=3)
    base = list(mf.DEFAULT_PDF)
    hp = 1e-4 * base[5]

    def sigma(a_u):
        pp = list(base)
        pp[5] = a_u
        return mf.Process(mf.Config(process="qg>ttxq", pdf_params=tuple(pp))).grad(n, iter_offset=3)[0][0]

    fd = (sigma(base[5] + hp) - sigma(base[5] - hp)) / (2 * hp)
    assert abs(fd - vals[2 + 5]) < 1e-8 * abs(vals[2 + 5]), (fd, vals[2 + 5])
