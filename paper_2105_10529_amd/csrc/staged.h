// Shared first stage of the multi-kernel integrands (HIP, gfx950): the
// kinematics, cuts and PDF factor of every point, and the compaction of the
// points that pass the cuts into a list, so that the amplitude kernels run
// on passing events only.  The list order depends on the order in which the
// waves reach the compaction; each event's result does not depend on its
// position in the list, and the weights land at the events' own indices.
#pragma once
#include <hip/hip_runtime.h>

#include "amp.h"
#include "launch.h"
#include "pipeline.h"

namespace mf {
namespace st {

// Kinematics, cuts and the event weight without |M|^2 (same steps and
// factors as event_weight for the g g channel).
template <int NG>
__device__ __forceinline__ bool kinematics(const DevCfg& c, const double* x, double& shat_k, V4<double>* gl,
                                           V4<double>& top, V4<double>& atop, double& wps) {
  const double x1 = x[0], x2 = x[1];
  const double shat = x1 * x2 * c.s;
  const double thr = 4.0 * c.mt * c.mt;
  bool ok = shat > thr;
  shat_k = ok ? shat : thr * (1.0 + 1e-3);
  wps = phase_space<double>(NG, x, shat_k, c.mt, gl, top, atop);
  ok = ok && (wps > 0.0);
  return ok && pass_cuts(c, NG, gl, 0.5 * log(x1 / x2));
}

static __global__ void k_st_zero(int* count) { *count = 0; }

// Every point: w = 0, wpre = the weight without |M|^2 (0 if the point fails
// threshold or cuts), and the passing points' indices appended to idx.
template <int NG>
__global__ void __launch_bounds__(BLOCK) k_st_select(DevCfg c, const double* __restrict__ u, int64_t n,
                                                     double* __restrict__ w, double* __restrict__ wpre,
                                                     int* __restrict__ idx, int* __restrict__ count) {
  const int64_t e0 = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  const bool live = e0 < n;
  const int64_t e = live ? e0 : n - 1;
  double x[MAXD];
#pragma unroll
  for (int j = 0; j < MAXD; ++j)
    if (j < c.ndim) x[j] = u[(int64_t)j * n + e];
  double shat_k, wps;
  V4<double> gl[NG], top, atop;
  bool ok = kinematics<NG>(c, x, shat_k, gl, top, atop, wps);
  const double tq = c.dyn_scale ? q_position(half_ht<NG>(c.mt, top, atop, gl)) : 0.0;
  const double pre = c.norm / (2.0 * shat_k * x[0] * x[1]) * wps *
                     (pdf_at(c, c.pdfc, 0, x_position(c, x[0]), tq) * pdf_at(c, c.pdfc, 0, x_position(c, x[1]), tq));
  ok = ok && live && isfinite(pre) && pre != 0.0;
  if (live) {
    w[e] = 0.0;
    wpre[e] = ok ? pre : 0.0;
  }
  // compaction: one atomic per wave, ranks from the ballot
  const unsigned long long b = __ballot(ok);
  const int lane = threadIdx.x & 63;
  const int rank = __popcll(b & ((1ull << lane) - 1ull));
  int base = 0;
  if (lane == 0 && b != 0ull) base = atomicAdd(count, __popcll(b));
  base = __shfl(base, 0);
  if (ok) idx[base + rank] = (int)e;
}

}  // namespace st
}  // namespace mf
