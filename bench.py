"""Benchmark of the on-device VEGAS integration of the LO integrand.

Headline workload (one "step" = one VEGAS iteration = one pass of the whole
per-event pipeline over one batch): g g -> t t~ g g at sqrt(s) = 13 TeV,
m_t = 173 GeV, mu = m_t, each gluon pT > 20 GeV, |eta| < 2.5, Delta R > 0.4,
10-dimensional integrand, 50 bins per dimension, 1e8 Philox events per
iteration, amplitudes in FP32 with FP64 (double-double) sums.  Warmup
iterations adapt the grid; the timed iterations continue the same run.

Prints one JSON line: value = events/s of the whole job (inputs generated in
the kernel), and the metric's second half, the wall time from process
creation to a relative error of 1e-3 of FP32 amplitudes with the learned
(BF16 coupling-flow) proposal against plain FP64 VEGAS (and FP32 VEGAS), for
three seeds, with the time inside the iteration that crosses the target
interpolated.  The roofline entry prices the selection + fused per-event
kernels' algorithmic FP32 flops (the emitted amplitude recursion and colour
form, counted statically, for each event that passes the cuts: only those
reach the matrix element) against the MI355X FP32 vector peak, using the
kernel time the library measures with HIP events on the call's stream.  The
CPU baseline times the FP64 oracle on a bounded sample of the same
adapted-grid events.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "events/s per MI355X and time to 1e-3 rel. error: FP32+flow vs FP64 VEGAS"
FP64_VECTOR_PEAK = 78.6e12  # MI355X FP64 vector FLOP/s (256 CUs x 64 FMA lanes x 2 flops x 2.4 GHz)
FP32_VECTOR_PEAK = 157.3e12  # MI355X FP32 vector FLOP/s (published; needs packed FP32 instructions)
FP32_UNPACKED_PEAK = 78.6e12  # the same chip without packed FP32 (this build's device code uses none)
HEADLINE_EVENTS = 100_000_000
EVENTS = 10_000_000
SEEDS = (2105105290, 2105105291, 2105105292)
TARGET = 1e-3
# HBM bytes of the kernel pair k_select<2> + k_vegas<2,0,float> per kept
# event (the list entry, written and read, and the fused kernel's register
# spill), from rocprofv3 FETCH_SIZE and WRITE_SIZE runs scaled by a 1 GiB copy
# calibration (profiles/traffic_k_vegas_gg_ttgg_fp32_1e8.md); the same in
# every iteration measured, so the traffic of a launch is this times its kept
# events.
TTGG_TRAFFIC_BYTES_PER_KEPT_EVENT = 1071.0
# the same for k_select<1> + k_vegas<1,0,double> at 1e7 events
# (profiles/traffic_k_vegas_gg_ttg_fp64_1e7.md)
TTG_TRAFFIC_BYTES = 52.7e6


def flops_per_event(m: int) -> int:
    sys.path.insert(0, os.path.join(ROOT, "paper_2105_10529_amd", "gen"))
    import gen_me

    return gen_me.flop_count(m)["total"]


def ttgg_config(prec: str, seed: int = SEEDS[0], **kw):
    import paper_2105_10529_amd as mf

    return mf.Config(process="gg>ttxgg", precision=prec, dr_min=0.4, seed=seed, **kw)


def interpolated_time(r, t_call: float, target: float = TARGET, prior=None):
    """Time (from process creation) and events at which the combined relative
    error of a run first reaches `target`, with the crossing iteration
    interpolated: inside it both the inverse variance and the wall time are
    taken to grow linearly with its events.  r: an IntegrationResult with
    per-iteration estimates and end times (seconds from the start of the
    call, which started t_call after process creation); prior: an earlier
    estimate combined first.  Returns (seconds, iterations as a fraction) or
    (None, None) if the run never reached the target."""
    I = np.asarray(r.iter_integral, float)
    E = np.asarray(r.iter_error, float)
    T = np.asarray(r.iter_seconds, float)
    w = np.where(E > 0, 1.0 / np.maximum(E, 1e-300) ** 2, 0.0)
    W0 = WI0 = 0.0
    if prior is not None and prior.error > 0:
        W0 = 1.0 / prior.error**2
        WI0 = prior.integral * W0
    W = W0 + np.cumsum(w)
    mean = (WI0 + np.sum(I * w)) / W[-1]
    need = 1.0 / (target * abs(mean)) ** 2
    if W0 >= need:
        return t_call, 0.0
    k = int(np.argmax(W >= need)) if np.any(W >= need) else -1
    if k < 0:
        return None, None
    Wp = W0 if k == 0 else W[k - 1]
    f = (need - Wp) / (W[k] - Wp)
    tp = 0.0 if k == 0 else T[k - 1]
    return t_call + tp + f * (T[k] - tp), k + f


def _spread(xs):
    xs = [float(x) for x in xs]
    return {"median": float(np.median(xs)), "min": min(xs), "max": max(xs), "per_seed": xs}


def _eff(stats: dict) -> dict:
    return {"mean_over_max": stats["mean"] / stats["max"], "mean_over_q999": stats["mean"] / stats["quantile"]}


def _load_kernels(process: str, precisions, helicity: int = 0) -> None:
    """Run every kernel of the VEGAS and flow pipelines once (untimed), so that
    no timing includes one-time code-object loading."""
    import torch

    import paper_2105_10529_amd as mf

    for prec in precisions:
        w = mf.Process(mf.Config(process=process, precision=prec, dr_min=0.4, helicity=helicity))
        w.integrate(2, 20_000, adapt=True)
        if prec == "fp32":
            wf = mf.Flow(w.ndim, max_batch=1024)
            w.train_flow_online(wf, 2, batch=1024, loss="variance", flow_mix=0.2)
            w.integrate(1, 20_000, adapt=False, flow=wf, flow_mix=0.2)
            w.integrate(2, 20_000, adapt=False, flow=wf, flow_mix=0.2, fallback_rel_var=1e-30)
            mf.weight_stats(w.weights(0, 20_000, flow=wf, flow_mix=0.2)[0])
            del wf
        del w
    torch.cuda.synchronize()


def learned_vs_vegas(process: str = "gg>ttxgg", precisions=("fp64", "fp32"), seeds=SEEDS,
                     vegas_events: int = 10_000_000, flow_iter_events: int = 4_000_000, steps: int = 15,
                     batch: int = 65536, lr: float = 5e-3, helicity: int = 0, eval_events: int = 10_000_000,
                     long_steps: int = 60, warm_iters: int = 5, warm_events: int = 1_000_000) -> dict:
    """Wall time from process creation to a combined relative error of 1e-3,
    per seed, for plain VEGAS in each precision (iterations of vegas_events,
    the grid adapting after each) and for FP32 amplitudes with the learned
    proposal: VEGAS warm-up warm_iters x warm_events, `steps` on-policy variance-training
    steps of the flow (batch points per step from the flow mixed with 20%
    uniform points on the frozen grid; the batches are themselves unbiased
    estimates, pooled per 50 steps), then iterations of flow_iter_events
    points combined with that estimate, with plain VEGAS on the same frozen
    grid as the fallback when the flow's first iteration has a larger
    per-event relative variance than the last warm-up iteration of VEGAS.
    Times are given as measured to the iteration boundary and interpolated
    inside the crossing iteration.  For the first seed also the per-event
    relative variance and unweighting efficiency of both proposals on a fresh
    sample of eval_events on the final grid (and, with long_steps, of a flow
    trained that long, untimed)."""
    import torch

    import paper_2105_10529_amd as mf

    def cfg(prec, seed):
        return mf.Config(process=process, precision=prec, dr_min=0.4, helicity=helicity, seed=seed)

    _load_kernels(process, precisions, helicity)
    runs = {f"vegas_{p}": [] for p in precisions}
    runs["fp32_flow"] = []
    for si_, seed in enumerate(seeds):
        for prec in precisions:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p = mf.Process(cfg(prec, seed))
            t_call = time.perf_counter() - t0
            r = p.integrate(200, vegas_events, target_rel_err=TARGET, adapt=True)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            ti, k = interpolated_time(r, t_call)
            rec = {"seed": seed, "time_to_1e-3_s": t, "time_to_1e-3_interpolated_s": ti,
                   "iterations": r.n_iter_done, "iterations_interpolated": k,
                   "events_interpolated": None if k is None else k * vegas_events,
                   "integral_pb": r.integral, "error_pb": r.error,
                   "events_per_s": r.n_events_total / r.seconds}
            if si_ == 0 and eval_events:
                w, _ = p.weights(1 << 30, eval_events)
                st = mf.weight_stats(w)
                del w
                rec["relative_variance_per_event"] = st["relvar"]
                rec["unweighting"] = _eff(st)
            runs[f"vegas_{prec}"].append(rec)
            del p
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p = mf.Process(cfg("fp32", seed))
        warm = p.integrate(warm_iters, warm_events, adapt=True)
        torch.cuda.synchronize()
        t_warm = time.perf_counter() - t0
        # the VEGAS proposal's per-event relative variance on the frozen grid,
        # from the last warm-up iteration: (N - 1) sigma^2 / I^2
        rv_vegas = (warm_events - 1) * warm.iter_error[-1] ** 2 / warm.iter_integral[-1] ** 2
        f = mf.Flow(p.ndim, max_batch=batch, seed=seed)
        mix, group = 0.2, 50
        rel, est = p.train_flow_online(f, steps, batch=batch, lr=lr, loss="variance", flow_mix=mix,
                                       group_steps=group, target_rel_err=TARGET, with_estimate=True)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0 - t_warm
        r = None
        if est.time_to_target >= 0.0:
            t = ti = time.perf_counter() - t0
            k = 0.0
            final = est
        else:
            t_call = time.perf_counter() - t0
            r = p.integrate(200, flow_iter_events, target_rel_err=TARGET, adapt=False, flow=f, flow_mix=mix,
                            iter_offset=1 << 24, prior=est, fallback_rel_var=rv_vegas)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            ti, k = interpolated_time(r, t_call, prior=est)
            final = r
        rec = {"seed": seed, "time_to_1e-3_s": t, "time_to_1e-3_interpolated_s": ti,
               "warmup_s": t_warm, "training_s": t_train, "time_excluding_training_s": t - t_train,
               "training_steps": int(np.count_nonzero(rel)), "training_batch": batch, "learning_rate": lr,
               "training_estimate_pb": [est.integral, est.error],
               "iterations_after_training": 0 if r is None else r.n_iter_done,
               "iterations_after_training_interpolated": k,
               "integral_pb": final.integral, "error_pb": final.error,
               "vegas_warmup_relative_variance": rv_vegas,
               "flow_first_iteration_relative_variance": None if r is None else r.flow_rel_var,
               "fallback_to_vegas": None if r is None else bool(r.fallback_iter >= 0),
               "batch_relative_variance_first_last": [float(np.mean(rel[:5])), float(np.mean(rel[-10:]))]}
        if si_ == 0 and eval_events:
            wf, _ = p.weights(1 << 30, eval_events, flow=f, flow_mix=mix)
            sf = mf.weight_stats(wf)
            del wf
            wv, _ = p.weights(1 << 30, eval_events)
            sv = mf.weight_stats(wv)
            del wv
            rec.update({"relative_variance_per_event": sf["relvar"],
                        "relative_variance_per_event_vegas_same_grid": sv["relvar"],
                        "unweighting": _eff(sf), "unweighting_vegas_same_grid": _eff(sv)})
            if long_steps:
                fl = mf.Flow(p.ndim, max_batch=batch, seed=seed)
                p.train_flow_online(fl, long_steps, batch=batch, lr=lr, loss="variance", flow_mix=mix,
                                    iter_offset=1 << 26)
                w3, _ = p.weights(1 << 30, eval_events, flow=fl, flow_mix=mix)
                s3 = mf.weight_stats(w3)
                del w3, fl
                rec[f"trained_{long_steps}_steps"] = {"relative_variance_per_event": s3["relvar"],
                                                      "unweighting": _eff(s3)}
        runs["fp32_flow"].append(rec)
        del p, f
    out = {"process": process, "seeds": list(seeds), "vegas_events_per_iteration": vegas_events,
           "flow_events_per_iteration": flow_iter_events, "runs": runs, "time_to_1e-3_s": {},
           "time_to_1e-3_interpolated_s": {}}
    for key, lst in runs.items():
        out["time_to_1e-3_s"][key] = _spread([x["time_to_1e-3_s"] for x in lst])
        tis = [x["time_to_1e-3_interpolated_s"] for x in lst]
        out["time_to_1e-3_interpolated_s"][key] = _spread(tis) if all(v is not None for v in tis) else None
    return out


def ttggg_helicity_sampling(events: int = 4_000_000) -> dict:
    """g g -> t t~ g g g with one polarisation state per point (drawn by
    Philox, weight x 64) against the sum over the 64 states: events/s, the
    per-event relative variance of the weights on the same adapted grid, and
    the wall time of plain FP32 VEGAS to 1e-3 from process creation."""
    import torch

    import paper_2105_10529_amd as mf

    out = {}
    for mode in (0, 1):
        cfg = mf.Config(process="gg>ttxggg", precision="fp32", dr_min=0.4, helicity=mode)
        w = mf.Process(cfg)
        w.integrate(1, 200_000, adapt=True)  # load the kernels (untimed)
        del w
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p = mf.Process(cfg)
        r = p.integrate(200, events, target_rel_err=1e-3, adapt=True)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        wv, _ = p.weights(1 << 30, events)
        st = mf.weight_stats(wv)
        del wv
        t1 = time.perf_counter()
        r2 = p.integrate(3, events, adapt=False, iter_offset=1 << 20)
        dt = time.perf_counter() - t1
        out["summed_states" if mode == 0 else "sampled_state"] = {
            "time_to_1e-3_s": t, "iterations": r.n_iter_done, "events": r.n_events_total, "integral_pb": r.integral,
            "error_pb": r.error, "events_per_s": 3 * events / dt, "relative_variance_per_event": st["relvar"],
            "check_integral_pb": [r2.integral, r2.error]}
        del p
    return out


def ttggg_throughput(events: int = 4_000_000, iters: int = 3, prec: str = "fp32") -> dict:
    """g g -> t t~ g g g with FP32 (or FP64) amplitudes: events/s of staged VEGAS
    iterations (after a warm-up that adapts the grid), and the algorithmic
    FLOP/s of the amplitude and colour kernels from their statically counted
    flops per passing event and the kernel times of the iterations (HIP events
    around each iteration's integrand)."""
    import torch

    import paper_2105_10529_amd as mf

    sys.path.insert(0, os.path.join(ROOT, "paper_2105_10529_amd", "gen"))
    import gen_me

    fc = gen_me.amp_flop_count(5)
    p = mf.Process(mf.Config(process="gg>ttxggg", precision=prec, dr_min=0.4))
    p.integrate(3, 1_000_000, adapt=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = p.integrate(iters, events, adapt=True, iter_offset=3)
    dt = time.perf_counter() - t0
    passing = r.n_nonzero
    amp_flops = passing * fc["states"] * fc["amplitudes_per_state"]
    col_flops = passing * fc["states"] * fc["colour_per_state"]
    return {"events_per_s": iters * events / dt, "events_per_iteration": events, "cut_efficiency": passing /
            max(r.n_events_total, 1), "integral_pb": r.integral, "error_pb": r.error,
            "iteration_kernels_ms_avg": 1e3 * r.kernel_seconds / iters,
            "flops_per_passing_event": fc["total"],
            "algorithmic_tflops_whole_integrand": (amp_flops + col_flops) / r.kernel_seconds / 1e12,
            "amplitude_flops_per_passing_event": fc["states"] * fc["amplitudes_per_state"],
            "colour_flops_per_passing_event": fc["states"] * fc["colour_per_state"]}


def ttggg_flow_comparison(seeds=SEEDS[:1]) -> dict:
    """The learned-proposal comparison on g g -> t t~ g g g (13 dims; FP32
    amplitudes + flow against FP64 and FP32 VEGAS): iterations of 4e6 events, 60
    training steps of 65536 points (the fastest of 30/60 steps x 65536 and
    120 x 32768 measured; a learning rate of 1e-2 trained worse or diverged),
    flow iterations of 2e6 points, and a 150-step flow for the attainable
    variance; with the polarisation states summed and with one sampled state
    per point.  With sampled states the trained flow's variance exceeds the
    VEGAS proposal's on the same grid, and the fallback continues with VEGAS."""
    return {"summed_states": learned_vs_vegas("gg>ttxggg", ("fp64", "fp32"), seeds, 4_000_000, 2_000_000, 60,
                                              eval_events=4_000_000, long_steps=150),
            "sampled_state": learned_vs_vegas("gg>ttxggg", ("fp32",), seeds, 4_000_000, 4_000_000, 60,
                                              helicity=1, eval_events=4_000_000, long_steps=150)}


def ttg_dynamic_scale(events: int = EVENTS, iters: int = 10) -> dict:
    """The benchmark workload with the dynamic scale mu = H_T / 2 (full (x, Q)
    PDF interpolation per event): events/s and the cross section, beside the
    fixed scale mu = m_t."""
    import torch

    import paper_2105_10529_amd as mf

    out = {}
    for dyn in (False, True):
        p = mf.Process(mf.Config(process="gg>ttxg", dynamic_scale=dyn))
        p.integrate(2, events, adapt=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = p.integrate(iters, events, adapt=True, iter_offset=2)
        dt = time.perf_counter() - t0
        out["dynamic_mu_ht_half" if dyn else "fixed_mu_mt"] = {
            "events_per_s": iters * events / dt, "kernel_ms_per_iteration": 1e3 * r.kernel_seconds / iters,
            "integral_pb": r.integral, "error_pb": r.error}
    return out


def ttg_observables(events: int = EVENTS, iters: int = 10) -> dict:
    """Observable histograms filled during the benchmark workload (g g -> t t~ g
    FP64, 2 adapting warm-up iterations, then `iters` iterations of 1e7 events
    on the frozen grid): per-bin cross sections and errors of the top pT, the
    top-pair mass and the hardest-gluon pT, and the cost of the histograms
    (kernel time of the same iterations with and without them)."""
    import torch

    import paper_2105_10529_amd as mf

    spec = {"nbins": 20, "lo": (0.0, 345.0, 20.0), "hi": (600.0, 1545.0, 420.0)}
    p = mf.Process(mf.Config(process="gg>ttxg"))
    p.integrate(2, events, adapt=True)
    torch.cuda.synchronize()
    r0 = p.integrate(iters, events, adapt=False, iter_offset=2)
    r = p.integrate(iters, events, adapt=False, iter_offset=2, observables=spec)
    o = r.observables
    return {"names": list(o["names"]), "bin_edges": [list(map(float, e)) for e in o["edges"]],
            "sigma_pb": o["sigma_pb"].tolist(), "error_pb": o["error_pb"].tolist(),
            "integral_pb": r.integral, "error_total_pb": r.error, "events": o["events"],
            "kernel_ms_per_iteration_without": 1e3 * r0.kernel_seconds / iters,
            "kernel_ms_per_iteration_with": 1e3 * r.kernel_seconds / iters}


def fp32_subsample_check(n: int = 100_000) -> dict:
    """g g -> t t~ g g with FP32 amplitudes against the FP64 oracle on a
    subsample of n events of one VEGAS iteration on an adapted grid: the same
    Philox events through the same grid, per-event relative error of the
    weights and the relative error of their mean (the FP64 GPU path is
    reported beside it)."""
    import torch

    import oracle
    import paper_2105_10529_amd as mf

    p32 = mf.Process(mf.Config(process="gg>ttxgg", precision="fp32", dr_min=0.4))
    p32.integrate(5, 1_000_000, adapt=True)
    edges = torch.empty((10, 51), dtype=torch.float64, device="cuda")
    p32.integrate(1, 2, adapt=False, edges_out=edges, iter_offset=1 << 20)
    p64 = mf.Process(mf.Config(process="gg>ttxgg", precision="fp64", dr_min=0.4))
    p64.integrate(1, 2, adapt=False, edges_in=edges, iter_offset=1 << 20)
    it = 777
    w32 = p32.weights(it, n)[0].cpu().numpy()
    w64 = p64.weights(it, n)[0].cpu().numpy()
    E = edges.cpu().numpy()
    u = oracle.event_uniforms(n, 10, it, p32.cfg.seed, 0)
    xs = np.empty_like(u)
    jac = np.empty(n)
    for i in range(n):
        xs[i], jac[i], _ = oracle.vegas_map(E, u[i])
    t0 = time.perf_counter()
    ref = oracle.Oracle(oracle.Config(n_g=2, dr_min=0.4)).integrand(xs) * jac
    t_orc = time.perf_counter() - t0
    nz = ref != 0.0
    r32 = np.abs(w32[nz] - ref[nz]) / np.abs(ref[nz])
    r64 = np.abs(w64[nz] - ref[nz]) / np.abs(ref[nz])

    return {"events": n, "nonzero": int(nz.sum()), "same_zero_pattern": bool(np.array_equal(w32 != 0, nz)),
            "fp32_per_event_rel_err_max": float(r32.max()), "fp32_per_event_rel_err_median": float(np.median(r32)),
            "fp32_per_event_rel_err_q999": float(np.quantile(r32, 0.999)),
            "fp32_integral_rel_err": float(abs(w32.mean() - ref.mean()) / abs(ref.mean())),
            "fp64_per_event_rel_err_max": float(r64.max()),
            "fp64_integral_rel_err": float(abs(w64.mean() - ref.mean()) / abs(ref.mean())),
            "oracle_seconds": t_orc, "oracle_threads": oracle.max_threads()}


BF16_MFMA_PEAK = 2.5e15  # MI355X dense BF16 matrix-core FLOP/s


def flow_flops_per_event(masks) -> int:
    """Algorithmic flops of one pass of the coupling flow per event: the three
    dense layers of every coupling layer (2 flops per multiply-add, unpadded
    widths); the PQ transform is not counted."""
    h, no = 256, 65
    tot = 0
    for m in masks:
        da, db = int((~m).sum()), int(m.sum())
        tot += 2 * (da * h + h * h + h * db * no)
    return tot


def flow_roofline(n: int = 10_000_000) -> dict:
    """The flow's sampling direction (six coupling-layer launches) on n points
    of the 10-dimensional g g -> t t~ g g space with seeded random parameters,
    timed with HIP events on the launch stream; achieved BF16 matrix-core
    FLOP/s from the algorithmic count against the dense BF16 peak."""
    import torch

    import paper_2105_10529_amd as mf
    import seeded_inputs as si

    f = mf.Flow(10, max_batch=64)
    mk = f.masks()
    shapes = [(int((~m).sum()), 256, int(m.sum()) * 65) for m in mk]
    f.set_params(mf.Flow.flatten(si.flow_params(shapes, seed=7, scale_out=0.3)))
    g = torch.Generator(device="cuda")
    g.manual_seed(si.BASE_SEED)
    z = torch.rand((10, n), dtype=torch.float32, device="cuda", generator=g)
    f.inverse(z)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 3
    ev0.record(stream)
    for _ in range(reps):
        f.inverse(z, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    sec = ev0.elapsed_time(ev1) * 1e-3 / reps
    fpe = flow_flops_per_event(mk)
    return {"events": n, "ms_per_pass": 1e3 * sec, "ms_per_layer_launch": 1e3 * sec / len(mk),
            "events_per_s": n / sec, "flops_per_event": fpe, "achieved_tflops": fpe * n / sec / 1e12,
            "peak_tflops": BF16_MFMA_PEAK / 1e12, "frac": fpe * n / sec / BF16_MFMA_PEAK,
            "kernel": "k_coupling<true,false> (sampling direction, 64 events per workgroup)"}


def cpu_baseline(p32, iteration: int, target_seconds: float = 12.0) -> dict:
    """The FP64 oracle on the host cores, on the first events of one VEGAS
    iteration through the adapted grid of the timed run (the same Philox
    events the GPU draws for that iteration), sized from a short calibration
    run to take about target_seconds."""
    import torch

    import oracle

    edges = torch.empty((p32.ndim, 51), dtype=torch.float64, device="cuda")
    p32.integrate(1, 2, adapt=False, edges_out=edges, iter_offset=1 << 30)
    E = edges.cpu().numpy()
    orc = oracle.Oracle(oracle.Config(n_g=2, dr_min=0.4))
    orc.vegas_iteration(E, iteration, 500, p32.cfg.seed, purpose=0)  # thread start-up
    n = 20_000
    t0 = time.perf_counter()
    orc.vegas_iteration(E, iteration, n, p32.cfg.seed, purpose=0)
    dt = time.perf_counter() - t0
    n = int(max(n, min(5_000_000, n * target_seconds / max(dt, 1e-3))))
    t0 = time.perf_counter()
    S1, _, _, nz, _ = orc.vegas_iteration(E, iteration, n, p32.cfg.seed, purpose=0)
    dt = time.perf_counter() - t0
    w = p32.weights(iteration, n)[0]
    gpu_mean = float(w.sum().item()) / n
    return {"value": n / dt, "unit": "events/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"first {n} Philox events of VEGAS iteration {iteration} through the adapted grid of the "
                      f"timed run, gg->ttgg FP64 (Delta R > 0.4), OpenMP over events, {dt:.1f} s",
            "oracle_mean_pb": S1 / n, "gpu_fp32_mean_same_events_pb": gpu_mean,
            "relative_difference": abs(gpu_mean - S1 / n) / abs(S1 / n), "nonzero": nz}


def ttg_fp64(events: int = EVENTS, iters: int = 10, warmup: int = 2) -> dict:
    """g g -> t t~ g in FP64 (7 dims, gluon pT > 20 GeV, |eta| < 2.5):
    events/s of 1e7-event VEGAS iterations after an adapting warm-up, and the
    selection + fused kernels' algorithmic FP64 rate."""
    import torch

    import paper_2105_10529_amd as mf

    p = mf.Process(mf.Config(process="gg>ttxg", precision="fp64"))
    p.integrate(warmup, events, adapt=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = p.integrate(iters, events, adapt=True, iter_offset=warmup)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    fpe = flops_per_event(3)
    kavg = r.kernel_seconds / iters
    passing = r.n_nonzero / iters
    ach = fpe * passing / kavg
    return {"events_per_s": iters * events / dt, "kernel_ms_avg": 1e3 * kavg, "integral_pb": r.integral,
            "error_pb": r.error, "cut_efficiency": r.n_nonzero / max(r.n_events_total, 1),
            "roofline": {"bound": "alu", "achieved": ach / 1e12, "peak": FP64_VECTOR_PEAK / 1e12,
                         "unit": "TFLOP/s", "frac": ach / FP64_VECTOR_PEAK,
                         "traffic": TTG_TRAFFIC_BYTES if events == EVENTS else None,
                         "kernel": "k_select<1> + k_vegas<1,0,double>", "flops_per_passing_event": fpe}}


def colour_forms(iters: int = 2) -> dict:
    """A/B of the two colour forms of g g -> t t~ g g: the quadratic form in
    registers inside the fused kernel (colour_form 1, the default) against
    the staged form with the colour sum on the matrix cores (colour_form 2),
    events/s of VEGAS iterations after two adapting ones; FP32 at 1e8 and
    FP64 at 1e7 events per iteration."""
    import torch

    import paper_2105_10529_amd as mf

    out = {}
    for prec, n in (("fp32", HEADLINE_EVENTS), ("fp64", EVENTS)):
        for form in (1, 2):
            p = mf.Process(ttgg_config(prec, colour_form=form))
            p.integrate(2, EVENTS, adapt=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = p.integrate(iters, n, adapt=True, iter_offset=2)
            torch.cuda.synchronize()
            out[f"{prec}_colour_form_{form}"] = {"events_per_s": iters * n / (time.perf_counter() - t0),
                                                 "integral_pb": r.integral, "error_pb": r.error}
    return out


def ttgg_fp64_throughput(events: int = EVENTS, iters: int = 3) -> dict:
    """Plain FP64 VEGAS on g g -> t t~ g g (the baseline of the comparison):
    events/s of 1e7-event iterations after an adapting warm-up."""
    import torch

    import paper_2105_10529_amd as mf

    p = mf.Process(ttgg_config("fp64"))
    p.integrate(2, events, adapt=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = p.integrate(iters, events, adapt=True, iter_offset=2)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"events_per_s": iters * events / dt, "kernel_ms_avg": 1e3 * r.kernel_seconds / iters,
            "events_per_iteration": events}


def ttg_gradients() -> dict:
    """d sigma/d m_t on g g -> t t~ g at m_t = 171, 173, 175 GeV from 1e8
    pathwise-derivative events each, with a grid frozen from a VEGAS warm-up."""
    import torch

    import paper_2105_10529_amd as mf

    grads = {}
    for mt in (171.0, 173.0, 175.0):
        p = mf.Process(mf.Config(process="gg>ttxg", m_t=mt))
        p.integrate(5, 10_000_000, adapt=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        vals, errs = p.grad(100_000_000, iter_offset=100)
        dt = time.perf_counter() - t0
        grads[f"{mt:g}"] = {"sigma_pb": vals[0], "sigma_err": errs[0], "dsigma_dmt_pb_per_gev": vals[1],
                            "dsigma_dmt_err": errs[1], "dsigma_dAg_pb": vals[2], "events": 100_000_000,
                            "seconds": dt}
    return grads


def ttj_channels(events: int = EVENTS, iters: int = 5) -> dict:
    """The hadronic t t~ + jet rate at leading order by partonic channel (FP64,
    jet = the light parton with pT > 20 GeV, |eta| < 2.5): g g -> t t~ g,
    u u~ -> t t~ g, d d~ -> t t~ g and q g -> t t~ q (+ q~ g), each from
    3 adapting + `iters` iterations of 1e7 events; events/s of the latter."""
    import torch

    import paper_2105_10529_amd as mf

    out = {}
    total, var = 0.0, 0.0
    for proc in ("gg>ttxg", "uux>ttxg", "ddx>ttxg", "qg>ttxq"):
        p = mf.Process(mf.Config(process=proc))
        p.integrate(3, events, adapt=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = p.integrate(iters, events, adapt=True, iter_offset=3)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[proc] = {"sigma_pb": r.integral, "error_pb": r.error, "events_per_s": iters * events / dt}
        total += r.integral
        var += r.error ** 2
    out["total_pb"] = [total, var ** 0.5]
    return out


def extended() -> dict:
    """Longer measurements, not part of the default run (--extended)."""
    return {"ttg_observables": ttg_observables(), "ttg_dynamic_scale": ttg_dynamic_scale(),
            "ttggg_helicity_sampling": ttggg_helicity_sampling(), "ttggg_flow_vs_vegas": ttggg_flow_comparison(),
            "ttgg_flow_300_steps": learned_vs_vegas(precisions=("fp32",), seeds=SEEDS[:1], long_steps=300)}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--events", type=int, default=HEADLINE_EVENTS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-comparison", action="store_true",
                    help="skip the time-to-1e-3 comparison (profiling runs of the headline kernels)")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--extended", action="store_true",
                    help="also run observables, dynamic scale, g g -> t t~ g g g comparisons and a 300-step flow")
    ap.add_argument("--only", choices=("ttg", "flow", "ttggg", "comparison", "ttj", "ttgg64", "colour_forms"),
                    default=None,
                    help="only one measurement (profiling): ttg = g g -> t t~ g FP64 iterations, flow = the "
                         "coupling-flow sampling pass, ttggg = g g -> t t~ g g g throughput, comparison = the "
                         "time-to-1e-3 comparison, ttj = the t t~ + jet channels, ttgg64 = FP64 g g -> t t~ g g "
                         "throughput, colour_forms = the A/B of the two colour forms of g g -> t t~ g g")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (to calibrate HBM counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only (asked for --gpus {args.gpus}); "
              "run with --gpus 1", file=sys.stderr)
        return 2

    import torch

    import paper_2105_10529_amd as mf

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 8}), flush=True)
        return 0
    if args.only == "ttg":
        print(json.dumps({"ttg_fp64": ttg_fp64()}), flush=True)
        return 0
    if args.only == "flow":
        print(json.dumps({"flow_roofline": flow_roofline()}), flush=True)
        return 0
    if args.only == "ttggg":
        print(json.dumps({"ttggg_fp32": ttggg_throughput(),
                          "ttggg_fp64": ttggg_throughput(prec="fp64")}), flush=True)
        return 0
    if args.only == "colour_forms":
        print(json.dumps({"colour_forms": colour_forms()}), flush=True)
        return 0
    if args.only == "ttgg64":
        print(json.dumps({"ttgg_fp64": ttgg_fp64_throughput()}), flush=True)
        return 0
    if args.only == "ttj":
        print(json.dumps({"ttj_by_channel": ttj_channels()}), flush=True)
        return 0
    if args.only == "comparison":
        print(json.dumps({"comparison": learned_vs_vegas()}), flush=True)
        return 0

    # headline: g g -> t t~ g g, FP32 amplitudes, 1e8 events per VEGAS iteration
    p = mf.Process(ttgg_config("fp32"))
    stream = torch.cuda.current_stream()
    if args.warmup > 0:
        p.integrate(args.warmup, args.events, adapt=True, iter_offset=0, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    r = p.integrate(args.steps, args.events, adapt=True, iter_offset=args.warmup, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_s = ev0.elapsed_time(ev1) * 1e-3
    elapsed = max(wall, gpu_s)
    value = args.steps * args.events / elapsed
    print(f"# headline done: {value:.4g} events/s", file=sys.stderr, flush=True)

    fpe = flops_per_event(4)
    kernel_avg = r.kernel_seconds / args.steps
    passing = r.n_nonzero / args.steps  # events whose matrix element is evaluated, per launch
    achieved = fpe * passing / kernel_avg
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "gg->ttgg LO, 13 TeV, m_t=173 GeV, mu=m_t, each gluon pT>20 GeV |eta|<2.5, "
                        "Delta R>0.4; 10-dim VEGAS (50 bins/dim), 1e8 Philox events per iteration, FP32 "
                        "amplitudes with FP64 double-double sums; time to 1e-3: FP32 amplitudes + BF16 "
                        "coupling flow (VEGAS fallback) vs FP64 VEGAS",
            "events_per_step": args.events,
            "process": "gg>ttxgg",
            "parallelism": "single-gpu",
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": FP32_VECTOR_PEAK / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_VECTOR_PEAK,
            "peak_unpacked": FP32_UNPACKED_PEAK / 1e12,
            "frac_unpacked": achieved / FP32_UNPACKED_PEAK,
            "traffic": TTGG_TRAFFIC_BYTES_PER_KEPT_EVENT * passing if args.events == HEADLINE_EVENTS else None,
            "traffic_note": "HBM bytes per launch from FETCH_SIZE/WRITE_SIZE (copy-calibrated), 1071 B per kept "
                            "event: mostly the fused kernel's register spill; 0.1 TB/s, not the bound",
            "kernel": "k_select<2> + k_vegas<2,0,float> (cut selection, then the fused weight of the kept events)",
            "flops_per_event": fpe,
            "flops_per": "event that passes the cuts (the matrix element is evaluated for those only)",
            "evaluated_events_per_launch": passing,
            "kernel_ms_avg": 1e3 * kernel_avg,
        },
        "integral_pb": r.integral,
        "error_pb": r.error,
        "chi2_dof": r.chi2_dof,
        "cut_efficiency": r.n_nonzero / max(r.n_events_total, 1),
    }
    if not args.no_comparison:
        cmp_ = learned_vs_vegas()
        print("# comparison done", file=sys.stderr, flush=True)
        t = cmp_["time_to_1e-3_interpolated_s"]
        f64 = ttgg_fp64_throughput()
        out["time_to_1e-3_s"] = {
            "fp64_vegas": t["vegas_fp64"], "fp32_vegas": t["vegas_fp32"], "fp32_flow": t["fp32_flow"],
            "to_iteration_boundary": {k: v["median"] for k, v in cmp_["time_to_1e-3_s"].items()},
            "speedup_fp32_flow_vs_fp64_vegas": t["vegas_fp64"]["median"] / t["fp32_flow"]["median"],
            "seeds": list(SEEDS),
            "method": "wall time from process creation; inside the iteration that crosses 1e-3 the inverse "
                      "variance and the time are interpolated linearly in its events"}
        out["events_per_s"] = {"fp32_vegas": value, "fp64_vegas": f64["events_per_s"]}
        out["comparison"] = {
            "flow_fallback_to_vegas": [x["fallback_to_vegas"] for x in cmp_["runs"]["fp32_flow"]],
            "relative_variance_per_event": {
                "fp64_vegas": cmp_["runs"]["vegas_fp64"][0]["relative_variance_per_event"],
                "fp32_flow": cmp_["runs"]["fp32_flow"][0]["relative_variance_per_event"],
                "vegas_same_frozen_grid": cmp_["runs"]["fp32_flow"][0][
                    "relative_variance_per_event_vegas_same_grid"]},
            "unweighting_mean_over_max": {
                "fp64_vegas": cmp_["runs"]["vegas_fp64"][0]["unweighting"]["mean_over_max"],
                "fp32_flow": cmp_["runs"]["fp32_flow"][0]["unweighting"]["mean_over_max"]},
            "integral_pb": {k: [v[0]["integral_pb"], v[0]["error_pb"]] for k, v in cmp_["runs"].items()}}
    if not args.no_cpu_baseline:
        cb = cpu_baseline(p, iteration=777)
        if "time_to_1e-3_s" in out:
            ev = [x["events_interpolated"] for x in cmp_["runs"]["vegas_fp64"]]
            cb["time_to_1e-3_extrapolated_s"] = float(np.median(ev)) / cb["value"]
            cb["time_to_1e-3_note"] = ("extrapolation: the median number of events plain FP64 VEGAS needed on the "
                                       "GPU (same algorithm) divided by the oracle's events/s")
        out["cpu_baseline"] = cb
        print("# cpu baseline done", file=sys.stderr, flush=True)
    if not args.no_secondary:
        ttg = ttg_fp64()
        sub = fp32_subsample_check()
        fl = flow_roofline()
        g3 = ttggg_throughput()
        out["secondary"] = {
            "ttg_fp64": {k: ttg[k] for k in ("events_per_s", "kernel_ms_avg", "integral_pb", "error_pb")} | {
                "roofline_frac": ttg["roofline"]["frac"], "achieved_tflops": ttg["roofline"]["achieved"]},
            "ttgg_fp32_vs_oracle_1e5": {k: sub[k] for k in ("fp32_per_event_rel_err_max",
                                                             "fp32_per_event_rel_err_median",
                                                             "fp32_per_event_rel_err_q999", "fp32_integral_rel_err",
                                                             "fp64_per_event_rel_err_max", "same_zero_pattern")},
            "flow_sampling": {k: fl[k] for k in ("events_per_s", "ms_per_pass", "achieved_tflops", "frac")},
            "ttggg_fp32": {k: g3[k] for k in ("events_per_s", "cut_efficiency", "iteration_kernels_ms_avg",
                                               "algorithmic_tflops_whole_integrand")},
            "ttg_gradients_dsigma_dmt": {k: [v["dsigma_dmt_pb_per_gev"], v["dsigma_dmt_err"]]
                                         for k, v in ttg_gradients().items()},
            "ttj_by_channel": ttj_channels(),
        }
        print("# secondary done", file=sys.stderr, flush=True)
    if args.extended:
        out["extended"] = extended()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
