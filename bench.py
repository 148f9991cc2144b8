"""Benchmark of the on-device VEGAS integration of the LO integrand.

Workload (one "step" = one VEGAS iteration = one pass of the whole per-event
pipeline over one batch): g g -> t t~ g at sqrt(s) = 13 TeV, m_t = 173 GeV,
mu = m_t, gluon pT > 20 GeV and |eta| < 2.5, 7-dimensional integrand, 50 bins
per dimension, 1e7 Philox events per iteration, FP64 throughout.  Warmup
iterations adapt the grid; the timed iterations continue the same run.

Prints one JSON line (value = events/s of the whole job, inputs generated in
the kernel).  The roofline entry prices the fused per-event kernel's
algorithmic FP64 flops (the emitted amplitude recursion, counted statically,
for each event that passes the cuts: the kernel evaluates the matrix element
of those events only) against the MI355X FP64 vector peak, using the kernel
time the library measures with HIP events on the call's stream.  The CPU baseline times the
FP64 oracle on a bounded sample of the same event stream.
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
FP64_VECTOR_PEAK = 78.6e12  # MI355X FP64 vector FLOP/s (256 CUs x 128 FLOP/clk x 2.4 GHz)
EVENTS = 10_000_000
# HBM bytes per iteration of the kernel pair k_select<1> + k_vegas<1,0,double>
# at 1e7 events (29.9 + 37.0 MB), from rocprofv3 FETCH_SIZE and WRITE_SIZE
# runs scaled by a 1 GiB copy calibration
# (profiles/traffic_k_vegas_gg_ttg_fp64_1e7.md).  Set to None when those
# kernels change until the counters are taken again.
MEASURED_TRAFFIC_BYTES = 66.9e6


def flops_per_event(m: int) -> int:
    sys.path.insert(0, os.path.join(ROOT, "paper_2105_10529_amd", "gen"))
    import gen_me

    return gen_me.flop_count(m)["total"]


def cpu_baseline(seed: int, target_seconds: float = 15.0) -> dict:
    """The FP64 oracle on the host cores, on the first events of the same stream
    (sized from a short calibration run to take about target_seconds)."""
    import oracle

    orc = oracle.Oracle(oracle.Config(n_g=1))
    edges = oracle.uniform_edges(7)
    orc.vegas_iteration(edges, 0, 2000, seed, purpose=0)  # thread start-up
    n = 50_000
    t0 = time.perf_counter()
    orc.vegas_iteration(edges, 0, n, seed, purpose=0)
    dt = time.perf_counter() - t0
    n = int(max(n, min(10_000_000, n * target_seconds / max(dt, 1e-3))))
    t0 = time.perf_counter()
    orc.vegas_iteration(edges, 0, n, seed, purpose=0)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "events/s", "cores": oracle.max_threads(), "kind": "oracle",
            "sample": f"first {n} events of the same Philox stream (iteration 0) through a uniform grid, "
                      f"gg->ttg FP64, OpenMP over events, {dt:.1f} s"}


def _eff(stats: dict) -> dict:
    return {"mean_over_max": stats["mean"] / stats["max"], "mean_over_q999": stats["mean"] / stats["quantile"]}


def flow_comparison(n_iter_events: int = 10_000_000, eval_events: int = 10_000_000, steps: int = 30,
                    flow_iter_events: int = 4_000_000, vegas: bool = True, process: str = "gg>ttxgg",
                    precisions=("fp64", "fp32"), long_steps: int = 300, batch: int = 65536,
                    lr: float = 5e-3, helicity: int = 0) -> dict:
    """g g -> t t~ g g (or g g g; Delta R > 0.4): wall time from process
    creation to a relative error of 1e-3, for plain VEGAS in FP64 (where
    built), plain VEGAS with FP32 amplitudes, and FP32 amplitudes with the
    learned proposal: VEGAS warm-up
    5 x 1e6, `steps` on-policy variance-training steps of the flow (65536
    points per step, sampled from the flow mixed with 20% uniform points on
    the frozen grid), whose batches are themselves estimates of the integral
    (pooled per 50 steps and combined by inverse variance, stopping at 1e-3),
    then iterations of flow_iter_events points of the trained proposal
    combined with that estimate until 1e-3 (30 steps is the fastest setting
    measured to this target on g g -> t t~ g g; longer training lowers the
    variance further, which a second, untimed flow trained for long_steps
    steps shows).
    Also the per-event relative variance and the unweighting efficiency of
    each proposal on a fresh sample of eval_events with the final grid."""
    import torch

    import paper_2105_10529_amd as mf

    def cfg(prec):
        return mf.Config(process=process, precision=prec, dr_min=0.4, helicity=helicity)

    # load every kernel of the pipelines once (untimed), so that no timing
    # below includes one-time code-object loading
    for prec in precisions:
        w = mf.Process(cfg(prec))
        w.integrate(2, 20_000, adapt=True)
        if prec == "fp32":
            wf = mf.Flow(w.ndim, max_batch=1024)
            w.train_flow_online(wf, 2, batch=1024, loss="variance", flow_mix=0.2)
            w.integrate(1, 20_000, adapt=False, flow=wf, flow_mix=0.2)
            mf.weight_stats(w.weights(0, 20_000, flow=wf, flow_mix=0.2)[0])
            del wf
        del w
    torch.cuda.synchronize()
    res = {}
    for prec in (precisions if vegas else ()):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p = mf.Process(cfg(prec))
        r = p.integrate(100, n_iter_events, target_rel_err=1e-3, adapt=True)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        w, _ = p.weights(1 << 30, eval_events)
        st = mf.weight_stats(w)
        del w
        res[f"vegas_{prec}"] = {"time_to_1e-3_s": t, "iterations": r.n_iter_done, "events": r.n_events_total,
                                "integral_pb": r.integral, "error_pb": r.error,
                                "relative_variance_per_event": st["relvar"],
                                "unweighting": _eff(st)}
        del p
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p = mf.Process(cfg("fp32"))
    p.integrate(5, 1_000_000, adapt=True)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    f = mf.Flow(p.ndim, max_batch=batch)
    mix, group = 0.2, 50
    rel, est = p.train_flow_online(f, steps, batch=batch, lr=lr, loss="variance", flow_mix=mix,
                                   group_steps=group, target_rel_err=1e-3, with_estimate=True)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0 - t_warm
    if est.time_to_target >= 0.0:
        r = est
    else:
        r = p.integrate(100, flow_iter_events, target_rel_err=1e-3, adapt=False, flow=f, flow_mix=mix,
                        iter_offset=1 << 24, prior=est)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    wf, _ = p.weights(1 << 30, eval_events, flow=f, flow_mix=mix)
    sf = mf.weight_stats(wf)
    del wf
    wv, _ = p.weights(1 << 30, eval_events)
    sv = mf.weight_stats(wv)
    del wv
    # attainable variance: the same recipe trained for long_steps steps (untimed)
    f300 = mf.Flow(p.ndim, max_batch=batch)
    p.train_flow_online(f300, long_steps, batch=batch, lr=lr, loss="variance", flow_mix=mix,
                        iter_offset=1 << 26)
    w3, _ = p.weights(1 << 30, eval_events, flow=f300, flow_mix=mix)
    s3 = mf.weight_stats(w3)
    del w3, f300
    res["fp32_flow"] = {"time_to_1e-3_s": t, "time_excluding_training_s": t - t_train, "warmup_s": t_warm,
                        "training_s": t_train, "training_steps_done": int(np.count_nonzero(rel)),
                        "training_batch": batch, "learning_rate": lr,
                        "training_estimate_pb": [est.integral, est.error],
                        "training_events": est.n_events_total,
                        "iterations_after_training": r.n_iter_done if r is not est else 0,
                        "events_after_training": r.n_events_total if r is not est else 0,
                        "integral_pb": r.integral, "error_pb": r.error,
                        "batch_relative_variance_first_last": [float(np.mean(rel[:5])), float(np.mean(rel[-10:]))],
                        "relative_variance_per_event": sf["relvar"],
                        "relative_variance_per_event_vegas_same_grid": sv["relvar"],
                        "unweighting": _eff(sf), "unweighting_vegas_same_grid": _eff(sv),
                        f"trained_{long_steps}_steps": {"relative_variance_per_event": s3["relvar"],
                                                        "unweighting": _eff(s3)}}
    return res


FP32_VECTOR_PEAK = 157.3e12  # MI355X FP32 vector FLOP/s (published; packed FP32 instructions)
FP32_MATRIX_PEAK = 157.3e12  # MI355X FP32 matrix-core FLOP/s (dense)


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


def ttggg_throughput(events: int = 4_000_000, iters: int = 3) -> dict:
    """g g -> t t~ g g g with FP32 amplitudes: events/s of staged VEGAS
    iterations (after a warm-up that adapts the grid), and the algorithmic
    FLOP/s of the amplitude and colour kernels from their statically counted
    flops per passing event and the kernel times of the iterations (HIP events
    around each iteration's integrand)."""
    import torch

    import paper_2105_10529_amd as mf

    sys.path.insert(0, os.path.join(ROOT, "paper_2105_10529_amd", "gen"))
    import gen_me

    fc = gen_me.amp_flop_count(5)
    p = mf.Process(mf.Config(process="gg>ttxggg", precision="fp32", dr_min=0.4))
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


def ttggg_flow_comparison() -> dict:
    """The learned-proposal comparison on g g -> t t~ g g g (13 dims; FP32
    amplitudes, so FP32 VEGAS is the baseline): iterations of 4e6 events, 60
    training steps of 65536 points (the fastest of 30/60 steps x 65536 and
    120 x 32768 measured; a learning rate of 1e-2 trained worse or diverged),
    flow iterations of 2e6 points, and a 150-step flow for the attainable
    variance; with the polarisation states summed and with one sampled state
    per point.  With sampled states plain VEGAS is the faster method (the
    flow's grid is frozen after a warm-up whose variance is ~3x that of the
    fully adapted grid, and the state sampling adds noise to the training
    gradients; 30/60/120/200 steps measured 3.2/2.8/2.3/4.9 s against 0.9 s)."""
    return {"summed_states": flow_comparison(4_000_000, 4_000_000, 60, 2_000_000, process="gg>ttxggg",
                                             precisions=("fp32",), long_steps=150),
            "sampled_state": flow_comparison(4_000_000, 4_000_000, 60, 4_000_000, process="gg>ttxggg",
                                             precisions=("fp32",), long_steps=150, helicity=1)}


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


def secondary(seed_events: int) -> dict:
    """Bounded extra measurements on the same GPU (reported beside the main line).

    * g g -> t t~ g g (10 dims, Delta R > 0.4): events/s of the fused kernel
      with FP32 amplitudes (1e8 events per iteration) and with FP64 (1e7), and
      the wall time to 1e-3 relative error of plain VEGAS in each precision.
    * d sigma/d m_t on g g -> t t~ g at m_t = 171, 173, 175 GeV from 1e8
      pathwise-derivative events each, with a grid frozen from a VEGAS warm-up.
    """
    import torch

    import paper_2105_10529_amd as mf

    out = {}
    for prec, n in (("fp32", 100_000_000), ("fp64", 10_000_000)):
        p = mf.Process(mf.Config(process="gg>ttxgg", precision=prec, dr_min=0.4))
        p.integrate(2, min(n, 10_000_000), adapt=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = p.integrate(2, n, adapt=True, iter_offset=2)
        dt = time.perf_counter() - t0
        fresh = mf.Process(mf.Config(process="gg>ttxgg", precision=prec, dr_min=0.4))
        tt = fresh.integrate(40, 10_000_000, target_rel_err=1e-3, adapt=True)
        out[f"ttgg_{prec}"] = {
            "events_per_s": 2 * n / dt, "kernel_ms_avg": 1e3 * r.kernel_seconds / 2, "events_per_iteration": n,
            "integral_pb": r.integral, "error_pb": r.error,
            "time_to_1e-3_s": tt.time_to_target, "iterations_to_1e-3": tt.n_iter_done,
            "events_to_1e-3": tt.n_events_total, "integral_at_1e-3_pb": tt.integral, "error_at_1e-3_pb": tt.error,
        }
    out["ttgg_fp32_vs_oracle_subsample"] = fp32_subsample_check()
    out["ttgg_flow_vs_vegas"] = flow_comparison()
    out["ttg_observables"] = ttg_observables()
    out["ttg_dynamic_scale"] = ttg_dynamic_scale()
    out["ttggg_fp32"] = ttggg_throughput()
    out["ttggg_helicity_sampling"] = ttggg_helicity_sampling()
    out["ttggg_flow_vs_vegas"] = ttggg_flow_comparison()
    out["flow_roofline"] = flow_roofline()
    grads = {}
    for mt in (171.0, 173.0, 175.0):
        p = mf.Process(mf.Config(process="gg>ttxg", m_t=mt))
        p.integrate(5, 10_000_000, adapt=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        vals, errs = p.grad(100_000_000, iter_offset=100)
        dt = time.perf_counter() - t0
        grads[f"{mt:g}"] = {"sigma_pb": vals[0], "sigma_err": errs[0], "dsigma_dmt_pb_per_gev": vals[1],
                            "dsigma_dmt_err": errs[1], "dsigma_dtheta": list(map(float, vals[2:])),
                            "dsigma_dtheta_err": list(map(float, errs[2:])), "events": 100_000_000,
                            "seconds": dt}
    out["ttg_gradients"] = grads
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--events", type=int, default=EVENTS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--workload", choices=("ttg", "ttgg", "ttggg"), default="ttg",
                    help="ttg: g g -> t t~ g FP64 (the reported workload); ttgg, ttggg: g g -> t t~ g g (g) with "
                         "FP32 amplitudes (profiling runs)")
    ap.add_argument("--flow-only", action="store_true",
                    help="only run the g g -> t t~ g g learned-proposal comparison and the flow roofline (profiling)")
    ap.add_argument("--observables-only", action="store_true",
                    help="only run the g g -> t t~ g observable histograms (profiling)")
    ap.add_argument("--ttggg-only", action="store_true",
                    help="only run the g g -> t t~ g g g throughput and learned-proposal measurements (profiling)")
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
    if args.flow_only:
        print(json.dumps({"ttgg_flow_vs_vegas": flow_comparison(), "flow_roofline": flow_roofline()}), flush=True)
        return 0
    if args.observables_only:
        print(json.dumps({"ttg_observables": ttg_observables(), "ttg_dynamic_scale": ttg_dynamic_scale()}),
              flush=True)
        return 0
    if args.ttggg_only:
        print(json.dumps({"ttggg_fp32": ttggg_throughput(), "ttggg_helicity_sampling": ttggg_helicity_sampling(),
                          "ttggg_flow_vs_vegas": ttggg_flow_comparison()}), flush=True)
        return 0
    if args.workload in ("ttgg", "ttggg"):
        proc = "gg>ttx" + args.workload[2:]
        p = mf.Process(mf.Config(process=proc, precision="fp32", dr_min=0.4))
        if args.warmup:
            p.integrate(args.warmup, args.events, adapt=True)
        r = p.integrate(args.steps, args.events, adapt=True, iter_offset=args.warmup)
        print(json.dumps({"workload": f"{proc} fp32", "events_per_s": args.steps * args.events / r.seconds,
                          "kernel_ms_avg": 1e3 * r.kernel_seconds / args.steps,
                          "cut_efficiency": r.n_nonzero / max(r.n_events_total, 1),
                          "integral_pb": r.integral, "error_pb": r.error}), flush=True)
        return 0
    p = mf.Process(mf.Config(process="gg>ttxg", precision="fp64"))
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
    total_events = args.steps * args.events
    value = total_events / elapsed

    fpe = flops_per_event(3)
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
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "gg->ttg LO, 13 TeV, m_t=173 GeV, mu=m_t, gluon pT>20 GeV |eta|<2.5; "
                        "7-dim VEGAS (50 bins/dim), 1e7 Philox events per iteration, FP64",
            "events_per_step": args.events,
            "process": "gg>ttxg",
            "parallelism": "single-gpu",
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": FP64_VECTOR_PEAK / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_VECTOR_PEAK,
            "traffic": MEASURED_TRAFFIC_BYTES if args.events == EVENTS and MEASURED_TRAFFIC_BYTES else None,
            "traffic_unit": "bytes per iteration (HBM read + write of both kernels, counter-calibrated)",
            "kernel": "k_select<1> + k_vegas<1,0,double> (cut selection, then the fused weight of the kept events)",
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
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p.cfg.seed)
    if not args.no_secondary:
        out["secondary"] = secondary(args.events)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
