// Launcher table: the C ABI reaches the templated kernels of one process
// instance through these function pointers (one translation unit per
// instance keeps compilation parallel).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pipeline.h"

namespace mf {

constexpr int BLOCK = 256;
constexpr int WAVES = BLOCK / 64;
constexpr int MAX_BLOCKS = 2048;
constexpr int PART_HEAD = 8;  // S1 hi, S1 lo, S2 hi, S2 lo, nonzero, nonfinite, pad, pad
constexpr int GV = 10;        // w, dw/dm_t, dw/dtheta_0..7

// ---------------------------------------------------- compensated sums
struct KSum {
  double s, c;  // Kahan: the exact sum is approximately s - c
};
__device__ __forceinline__ void kadd(KSum& k, double v) {
  double y = v - k.c;
  double t = k.s + y;
  k.c = (t - k.s) - y;
  k.s = t;
}
// Error-free two-sum: a + b = s + e exactly.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
// Double-double accumulate (hi, lo) += v.
__device__ __forceinline__ void dd_add(double& hi, double& lo, double v) {
  double s, e;
  two_sum(hi, v, s, e);
  lo += e;
  two_sum(s, lo, hi, lo);
}

// Deterministic wave-wide sum of a double with error terms (xor butterfly of
// two-sums); every lane ends with the same (hi, lo).  The butterfly order is
// fixed and two-sum is exact, so the result does not depend on timing.
__device__ __forceinline__ void wave_sum_dd(double v, double& hi, double& lo) {
  double s = v, e = 0.0;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double so = __shfl_xor(s, off), eo = __shfl_xor(e, off);
    double t, err;
    two_sum(s, so, t, err);
    s = t;
    e = (e + eo) + err;
  }
  hi = s;
  lo = e;
}
// Per-wave double-double accumulator in LDS, updated identically by every
// lane of the wave (all lanes hold the same addend).
__device__ __forceinline__ void lds_dd_accumulate(double* acc, double hi, double lo) {
  double h = acc[0], l = acc[1];
  dd_add(h, l, hi);
  dd_add(h, l, lo);
  acc[0] = h;
  acc[1] = l;
}

// Observable histograms (k_observables): bins per observable and, per
// observable, the lower edge and nbins / (upper - lower edge).
constexpr int N_OBS = 3;
constexpr int MAX_OBS_BINS = 64;
struct ObsSpec {
  int nbins;
  double lo[N_OBS], scale[N_OBS];
};

struct Launchers {
  // false: VEGAS iterations go through the staged path (points kernel ->
  // integrand kernel -> accumulation kernel) instead of the fused kernel
  bool fused;
  // selection (k_select_points) then the weights of the kept points
  // (k_integrand); list/cnt/cap as for vegas
  void (*integrand)(const DevCfg&, const double*, int64_t, double*, int, int*, int*, int64_t, hipStream_t);
  void (*integrand_grad)(const DevCfg&, const double*, int64_t, double*, double*, int, hipStream_t);
  // selection (k_select) then the fused weight kernel (k_vegas) of one
  // iteration; list/cnt/cap: per-block event lists, [nblk][cap] and [nblk]
  void (*vegas)(const DevCfg&, const double*, uint64_t, int64_t, uint64_t, double*, int, int, size_t, int*, int*,
                int64_t, double*, hipStream_t);
  // observable histograms of the kept events of the last fused iteration
  // (their weights from vegas' wk output); per-block partial rows
  void (*observables)(const DevCfg&, const double*, uint64_t, uint64_t, const int*, const int*, int64_t,
                      const double*, const ObsSpec&, double*, int, hipStream_t);
  // selection (k_select) then the derivative estimator over the kept events
  void (*grad_vegas)(const DevCfg&, const double*, uint64_t, int64_t, uint64_t, double*, int, size_t, int*, int*,
                     int64_t, hipStream_t);
  // Multi-kernel integrand with a workspace held by the process handle
  // (*ws, created on first use, released with ws_free); used instead of
  // `integrand` when set.  Synchronises the stream (it reads the number of
  // events that pass the cuts).
  hipError_t (*integrand_ws)(const DevCfg&, const double*, int64_t, double*, void**, hipStream_t);
  void (*ws_free)(void*);
};

// One per built instance: g g -> t t~ + ng g in FP64 / FP32 amplitudes, and
// the quark channels in FP64.
Launchers launchers_gg0_f64();
Launchers launchers_gg0_f32();
Launchers launchers_gg1_f64();
Launchers launchers_gg1_f32();
Launchers launchers_gg2_f64();
Launchers launchers_gg2_f32();
Launchers launchers_uu_f64();
Launchers launchers_dd_f64();
// the quark channels with one more light parton (FP64)
Launchers launchers_uug_f64();
Launchers launchers_ddg_f64();
Launchers launchers_qg_f64();
Launchers launchers_gg3_f32();
Launchers launchers_gg3_f64();
// g g -> t t~ g g with the colour sum on the matrix cores (staged kernels)
Launchers launchers_gg2s_f32();
Launchers launchers_gg2s_f64();

}  // namespace mf
