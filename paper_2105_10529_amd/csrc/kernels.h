// Templated per-event kernels of the integrand library (HIP, gfx950),
// instantiated per process and amplitude precision in the inst_*.hip units
// and reached from the C ABI through the launcher table of launch.h.
#pragma once
#include <hip/hip_runtime.h>

#include "launch.h"
#include "pipeline.h"

namespace mf {
namespace {

// Block-chunked event loops: chunk `it` of this block covers events
// [chunk_base(it), chunk_base(it) + BLOCK).  Both quantities are uniform over
// the block and computed from scalars only.
__device__ __forceinline__ int64_t chunk_base(int64_t it) {
  return (int64_t)blockIdx.x * BLOCK + it * (int64_t)gridDim.x * BLOCK;
}
__device__ __forceinline__ int64_t chunks_of_block(int64_t n) {
  const int64_t b0 = (int64_t)blockIdx.x * BLOCK, stride = (int64_t)gridDim.x * BLOCK;
  return b0 < n ? (n - b0 + stride - 1) / stride : 0;
}

// -------------------------------------------------------------- integrand
// At caller-supplied points: k_select_points writes w = 0 for every point and
// lists, per block and in point order, the points that pass threshold and
// cuts; k_integrand evaluates the weights of the listed points only (full
// wavefronts of points that count, as in the fused iteration).
template <int NG>
__global__ void __launch_bounds__(BLOCK) k_select_points(DevCfg c, const double* __restrict__ u, int64_t n,
                                                         double* __restrict__ w, int* __restrict__ list,
                                                         int* __restrict__ cnt, int64_t cap) {
  __shared__ int wcount[WAVES];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int* out = list + (int64_t)blockIdx.x * cap;
  int qn = 0;
  const int64_t nchunk = chunks_of_block(n);
  for (int64_t it = 0; it < nchunk; ++it) {
    const int64_t e0 = chunk_base(it) + tid;
    const bool live = e0 < n;
    const int64_t e = live ? e0 : n - 1;
    double x[MAXD];
#pragma unroll
    for (int j = 0; j < MAXD; ++j)
      if (j < c.ndim) x[j] = u[(int64_t)j * n + e];
    const bool pass = event_passes<NG>(c, x) && live;
    if (live) w[e0] = 0.0;
    const unsigned long long b = __ballot(pass);
    if (lane == 0) wcount[wave] = __popcll(b);
    __syncthreads();
    int off = qn, total = 0;
#pragma unroll
    for (int v = 0; v < WAVES; ++v) {
      const int cv = wcount[v];
      off += v < wave ? cv : 0;
      total += cv;
    }
    if (pass) out[off + __popcll(b & ((1ull << lane) - 1ull))] = (int)e0;
    __syncthreads();
    qn += total;
  }
  if (tid == 0) cnt[blockIdx.x] = qn;
}

template <int NG, int CH, class RA>
__global__ void __launch_bounds__(BLOCK) k_integrand(DevCfg c, const double* __restrict__ u, int64_t n,
                                                     double* __restrict__ w, const int* __restrict__ list,
                                                     const int* __restrict__ cnt, int64_t cap) {
  const int* mine_list = list + (int64_t)blockIdx.x * cap;
  const int nsel = __builtin_amdgcn_readfirstlane(cnt[blockIdx.x]);
  const int64_t nchunk = (nsel + BLOCK - 1) / BLOCK;
  for (int64_t it = 0; it < nchunk; ++it) {
    const int64_t j0 = it * BLOCK + threadIdx.x;
    const bool live = j0 < nsel;
    const int64_t e = mine_list[live ? j0 : 0];  // idle lanes recompute the block's first point
    double x[MAXD];
#pragma unroll
    for (int j = 0; j < MAXD; ++j)
      if (j < c.ndim) x[j] = u[(int64_t)j * n + e];
    EventOut<double> r = event_weight<NG, CH, RA, double>(c, x, c.mt, c.pdfc);
    const double v = isfinite(r.w) ? r.w : 0.0;
    if (live) w[e] = v;
  }
}

// Derivatives of the event weight: m_t by a dual number through phase space
// and amplitudes, plus the scale derivative of the PDFs when mu = m_t; PDF
// parameters through the collapsed derivative tables.
template <int NG, int CH, class RA>
__device__ __forceinline__ void grad_event(const DevCfg& c, const double* x, double& w, double* dw) {
  EventOut<Dual<double>> r = event_weight<NG, CH, RA, Dual<double>>(c, x, Dual<double>(c.mt, 1.0), c.pdfc);
  w = r.w.v;
  for (int k = 0; k < 9; ++k) dw[k] = 0.0;
  dw[0] = r.w.d;  // r1, r2 and w are zero for an event that fails, so every term below is 0
  if constexpr (CH == 0) {
    double f1 = hermite_x(c.pdfc, r.t1), f2 = hermite_x(c.pdfc, r.t2);
    if (c.mu_is_mt) dw[0] += r.r1.v * (hermite_x(c.pdfd, r.t1) * f2 + f1 * hermite_x(c.pdfd, r.t2));
    for (int k = 0; k < 5; ++k) {
      const double* T = c.pdft + k * NXK;
      dw[1 + k] = r.r1.v * (hermite_x(T, r.t1) * f2 + f1 * hermite_x(T, r.t2));
    }
  } else if constexpr (CH == 3) {
    // w = r1 (u1 + d1) g2 + r2 g1 (u2 + d2) + r3 2 ub1 g2 + r4 g1 2 ub2
    const double* G = c.pdfc;
    const double *U = c.pdfc + NXK, *D = c.pdfc + 2 * NXK, *A = c.pdfc + 3 * NXK;
    const double g1 = hermite_x(G, r.t1), g2 = hermite_x(G, r.t2);
    const double q1 = hermite_x(U, r.t1) + hermite_x(D, r.t1), q2 = hermite_x(U, r.t2) + hermite_x(D, r.t2);
    const double a1 = 2.0 * hermite_x(A, r.t1), a2 = 2.0 * hermite_x(A, r.t2);
    if (c.mu_is_mt) {
      const double* dG = c.pdfd;
      const double *dU = c.pdfd + NXK, *dD = c.pdfd + 2 * NXK, *dA = c.pdfd + 3 * NXK;
      const double dg1 = hermite_x(dG, r.t1), dg2 = hermite_x(dG, r.t2);
      const double dq1 = hermite_x(dU, r.t1) + hermite_x(dD, r.t1), dq2 = hermite_x(dU, r.t2) + hermite_x(dD, r.t2);
      const double da1 = 2.0 * hermite_x(dA, r.t1), da2 = 2.0 * hermite_x(dA, r.t2);
      dw[0] += r.r1.v * (dq1 * g2 + q1 * dg2) + r.r2.v * (dg1 * q2 + g1 * dq2) + r.r3.v * (da1 * g2 + a1 * dg2) +
               r.r4.v * (dg1 * a2 + g1 * da2);
    }
    for (int k = 0; k < 5; ++k) {
      const double* T = c.pdft + k * NXK;
      const double t1 = hermite_x(T, r.t1), t2 = hermite_x(T, r.t2);
      dw[1 + k] = r.r1.v * q1 * t2 + r.r2.v * t1 * q2 + r.r3.v * a1 * t2 + r.r4.v * t1 * a2;
    }
    const double *TU = c.pdft + 5 * NXK, *TD = c.pdft + 6 * NXK, *TA = c.pdft + 7 * NXK;
    dw[6] = r.r1.v * hermite_x(TU, r.t1) * g2 + r.r2.v * g1 * hermite_x(TU, r.t2);
    dw[7] = r.r1.v * hermite_x(TD, r.t1) * g2 + r.r2.v * g1 * hermite_x(TD, r.t2);
    dw[8] = r.r3.v * 2.0 * hermite_x(TA, r.t1) * g2 + r.r4.v * g1 * 2.0 * hermite_x(TA, r.t2);
  } else {
    const int fq = CH == 1 ? 1 : 2;
    const double* Q = c.pdfc + fq * NXK;
    const double* A = c.pdfc + 3 * NXK;
    double q1 = hermite_x(Q, r.t1), a2 = hermite_x(A, r.t2), a1 = hermite_x(A, r.t1), q2 = hermite_x(Q, r.t2);
    if (c.mu_is_mt) {
      const double* dQ = c.pdfd + fq * NXK;
      const double* dA = c.pdfd + 3 * NXK;
      dw[0] += r.r1.v * (hermite_x(dQ, r.t1) * a2 + q1 * hermite_x(dA, r.t2)) +
               r.r2.v * (hermite_x(dA, r.t1) * q2 + a1 * hermite_x(dQ, r.t2));
    }
    const double* TQ = c.pdft + (CH == 1 ? 5 : 6) * NXK;
    const double* TA = c.pdft + 7 * NXK;
    dw[CH == 1 ? 6 : 7] = r.r1.v * (hermite_x(TQ, r.t1) * a2) + r.r2.v * (a1 * hermite_x(TQ, r.t2));
    dw[8] = r.r1.v * (q1 * hermite_x(TA, r.t2)) + r.r2.v * (hermite_x(TA, r.t1) * q2);
  }
}

template <int NG, int CH, class RA>
__global__ void __launch_bounds__(BLOCK) k_integrand_grad(DevCfg c, const double* __restrict__ u, int64_t n,
                                                          double* __restrict__ w, double* __restrict__ dw) {
  const int64_t nchunk = chunks_of_block(n);
  for (int64_t it = 0; it < nchunk; ++it) {
    const int64_t e0 = chunk_base(it) + threadIdx.x;
    const bool live = e0 < n;
    const int64_t e = live ? e0 : n - 1;
    double x[MAXD];
#pragma unroll
    for (int j = 0; j < MAXD; ++j)
      if (j < c.ndim) x[j] = u[(int64_t)j * n + e];
    double ww, d[9];
    grad_event<NG, CH, RA>(c, x, ww, d);
    bool ok = isfinite(ww);
    for (int k = 0; k < 9; ++k) ok = ok && isfinite(d[k]);
    if (live) {
      if (w) w[e] = ok ? ww : 0.0;
      for (int k = 0; k < 9; ++k) dw[(int64_t)k * n + e] = ok ? d[k] : 0.0;
    }
  }
}

// ----------------------------------------------------- event selection
// Stage 1 of a VEGAS iteration: every event of the block's chunks (the same
// interleaved chunks as the fused kernel) is drawn, mapped and tested for
// threshold and cuts (kinematics only); the indices of the events that pass
// are written, in event order, to the block's own slice list[b * cap ...]
// and their number to cnt[b].  The fused kernel then evaluates the weight of
// those events only, on full wavefronts; events that fail contribute zero
// to every sum and histogram.
template <int NG>
__global__ void __launch_bounds__(BLOCK) k_select(DevCfg c, const double* __restrict__ edges_g, uint64_t iter,
                                                  int64_t N, uint64_t seed, int* __restrict__ list,
                                                  int* __restrict__ cnt, int64_t cap) {
  extern __shared__ double lds[];
  __shared__ int wcount[WAVES];
  const int d = c.ndim, nb = c.nb;
  double* edges = lds;  // d*(nb+1)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < d * (nb + 1); i += BLOCK) edges[i] = edges_g[i];
  __syncthreads();
  int* out = list + (int64_t)blockIdx.x * cap;
  int qn = 0;
  const int64_t nchunk = chunks_of_block(N);
  for (int64_t it = 0; it < nchunk; ++it) {
    const int64_t e0 = chunk_base(it) + tid;
    const bool live = e0 < N;
    double y[MAXD], x[MAXD];
    event_uniforms((uint64_t)(live ? e0 : N - 1), iter, seed, 0, d, y);
    double jac = 1.0;
#pragma unroll
    for (int j = 0; j < MAXD; ++j)
      if (j < d) {
        int bin;
        x[j] = vegas_map_dim(edges + j * (nb + 1), nb, y[j], bin, jac);
      }
    const bool pass = event_passes<NG>(c, x) && live;
    const unsigned long long b = __ballot(pass);
    if (lane == 0) wcount[wave] = __popcll(b);
    __syncthreads();
    int off = qn, total = 0;
#pragma unroll
    for (int v = 0; v < WAVES; ++v) {
      const int cv = wcount[v];
      off += v < wave ? cv : 0;
      total += cv;
    }
    if (pass) out[off + __popcll(b & ((1ull << lane) - 1ull))] = (int)e0;
    __syncthreads();
    qn += total;
  }
  if (tid == 0) cnt[blockIdx.x] = qn;
}

// ----------------------------------------------------- fused VEGAS iteration
// Stage 2: the weights of the events k_select kept for this block (chunks of
// BLOCK list entries; the last chunk's idle lanes recompute the block's first
// event with the weight masked).
template <int NG, int CH, class RA>
__global__ void __launch_bounds__(BLOCK) k_vegas(DevCfg c, const double* __restrict__ edges_g, uint64_t iter,
                                                 int64_t N, uint64_t seed, double* __restrict__ partials,
                                                 int pstride, const int* __restrict__ list,
                                                 const int* __restrict__ cnt, int64_t cap,
                                                 double* __restrict__ wk) {
  extern __shared__ double lds[];
  const int d = c.ndim, nb = c.nb;
  double* edges = lds;                             // d*(nb+1)
  double* pdf = edges + d * (nb + 1);              // 4*196
  double* hist = pdf + 4 * NXK;                    // WAVES*d*nb
  double* dummy = hist + WAVES * d * nb;           // WAVES*nb: rows for lanes >= d
  double* wacc = dummy + WAVES * nb;               // WAVES*4 compensated sums
  double* w2s = wacc + WAVES * 4;                  // BLOCK
  double* jac_s = w2s + BLOCK;                     // BLOCK
  double* xs = jac_s + BLOCK;                      // d*BLOCK mapped points
  unsigned char* bins_s = (unsigned char*)(xs + d * BLOCK);  // d*BLOCK
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < d * (nb + 1); i += BLOCK) edges[i] = edges_g[i];
  for (int i = tid; i < 4 * NXK; i += BLOCK) pdf[i] = c.pdfc[i];
  for (int i = tid; i < WAVES * (d + 1) * nb + WAVES * 4; i += BLOCK) hist[i] = 0.0;
  __syncthreads();
  DevCfg cl = c;
  cl.pdfc = pdf;
  // Nothing per lane is carried from one event chunk to the next: sums go to
  // per-wave LDS accumulators after a deterministic wave reduction, counts are
  // ballots (wave-uniform scalars).
  double* acc = wacc + wave * 4;  // S1 (hi, lo), S2 (hi, lo)
  unsigned long long nnz = 0, nbad = 0;
  double* my_hist = hist + wave * d * nb;
  // The chunk loop is controlled by block-uniform scalars (the length of the
  // block's list), so its counter lives in scalar registers and is not
  // exposed to vector-register spills inside the divergent per-event code.
  const int* mine_list = list + (int64_t)blockIdx.x * cap;
  const int nsel = __builtin_amdgcn_readfirstlane(cnt[blockIdx.x]);
  const int64_t nchunk = (nsel + BLOCK - 1) / BLOCK;
  for (int64_t it = 0; it < nchunk; ++it) {
    const int64_t j0 = it * BLOCK + tid;
    const bool live = j0 < nsel;
    const int64_t e = mine_list[live ? j0 : 0];
    {
      // map the uniforms and stage the bin indices and the Jacobian in LDS
      // before the amplitude, so no per-lane value is live across it
      int bins[MAXD];
      double y[MAXD];
      event_uniforms((uint64_t)e, iter, seed, 0, d, y);
      double jac = 1.0;
#pragma unroll
      for (int j = 0; j < MAXD; ++j)
        if (j < d) xs[j * BLOCK + tid] = vegas_map_dim(edges + j * (nb + 1), nb, y[j], bins[j], jac);
#pragma unroll
      for (int j = 0; j < MAXD; ++j)
        if (j < d) bins_s[j * BLOCK + tid] = (unsigned char)bins[j];
      jac_s[tid] = jac;
    }
    asm volatile("" ::: "memory");
    double x[MAXD];
#pragma unroll
    for (int j = 0; j < MAXD; ++j)
      if (j < d) x[j] = xs[j * BLOCK + tid];
    EventOut<double> r = event_weight<NG, CH, RA, double>(cl, x, c.mt, pdf);
    asm volatile("" ::: "memory");
    double w = r.w * jac_s[tid];
    const bool finite = isfinite(w);
    nbad += __popcll(__ballot(live && !finite));
    w = (live && finite) ? w : 0.0;
    nnz += __popcll(__ballot(w != 0.0));
    if (wk != nullptr && live) wk[(int64_t)blockIdx.x * cap + j0] = w;  // for the observable histograms
    {
      double h1, l1, h2, l2;
      wave_sum_dd(w, h1, l1);
      wave_sum_dd(w * w, h2, l2);
      lds_dd_accumulate(acc, h1, l1);
      lds_dd_accumulate(acc + 2, h2, l2);
    }
    // stage this wave's 64 weights, then bin them in event order
    w2s[tid] = w * w;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    {
      // every lane runs the binning loop (no divergent region in the event
      // loop); lanes >= d update a scratch row of their wave
      const bool mine = lane < d;
      const unsigned char* bj = bins_s + (mine ? lane : 0) * BLOCK + wave * 64;
      const double* ws = w2s + wave * 64;
      double* hj = mine ? my_hist + lane * nb : dummy + wave * nb;
      for (int k = 0; k < 64; ++k) hj[bj[k]] += ws[k];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  __syncthreads();
  // combine the wave histograms in wave order, then the compensated sums in
  // thread order (a fixed order: the partials are bitwise reproducible)
  double* p = partials + (int64_t)blockIdx.x * pstride;
  for (int i = tid; i < d * nb; i += BLOCK) {
    double h = 0.0;
    for (int v = 0; v < WAVES; ++v) h += hist[v * d * nb + i];
    p[PART_HEAD + i] = h;
  }
  __syncthreads();
  // counts: wave-uniform per wave; combine the four waves in order
  unsigned long long* ci = (unsigned long long*)w2s;
  if (lane == 0) {
    ci[wave] = nnz;
    ci[WAVES + wave] = nbad;
  }
  __syncthreads();
  if (tid == 0) {
    double acc_hi[2] = {0.0, 0.0}, acc_lo[2] = {0.0, 0.0};
    unsigned long long tn = 0, tb = 0;
    for (int v = 0; v < WAVES; ++v) {
      dd_add(acc_hi[0], acc_lo[0], wacc[4 * v + 0]);
      dd_add(acc_hi[0], acc_lo[0], wacc[4 * v + 1]);
      dd_add(acc_hi[1], acc_lo[1], wacc[4 * v + 2]);
      dd_add(acc_hi[1], acc_lo[1], wacc[4 * v + 3]);
      tn += ci[v];
      tb += ci[WAVES + v];
    }
    p[0] = acc_hi[0];
    p[1] = acc_lo[0];
    p[2] = acc_hi[1];
    p[3] = acc_lo[1];
    p[4] = (double)tn;
    p[5] = (double)tb;
  }
}

// ------------------------------------------------- observable histograms
// Weighted histograms of three observables of the kept events of one fused
// iteration (after k_vegas wrote their weights wk, in list order): 0 = top
// transverse momentum, 1 = invariant mass of the top pair, 2 = transverse
// momentum of the hardest gluon (absent without final gluons).  All three
// are invariant under the longitudinal boost, so they are taken from the
// partonic centre-of-mass momenta of the phase-space map.  Per bin the sum
// of w and of w^2; bin k = floor((v - lo) scale), kept for 0 <= k < nbins.
// One wave's 64 events are staged in LDS and binned by lanes 0..2 (one
// observable each) in event order, so the block partials are reproducible.
template <int NG>
__global__ void __launch_bounds__(BLOCK) k_observables(DevCfg c, const double* __restrict__ edges_g, uint64_t iter,
                                                       uint64_t seed, const int* __restrict__ list,
                                                       const int* __restrict__ cnt, int64_t cap,
                                                       const double* __restrict__ wk, ObsSpec o,
                                                       double* __restrict__ opart) {
  extern __shared__ double lds[];
  const int d = c.ndim, nb = c.nb, onb = o.nbins;
  const int W = N_OBS * onb * 2;
  double* edges = lds;                       // d*(nb+1)
  double* hw = edges + d * (nb + 1);         // [WAVES][N_OBS][onb][2]
  double* ws = hw + WAVES * W;               // [BLOCK] staged weights
  int* ks = (int*)(ws + BLOCK);              // [N_OBS][BLOCK] staged bins
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < d * (nb + 1); i += BLOCK) edges[i] = edges_g[i];
  for (int i = tid; i < WAVES * W; i += BLOCK) hw[i] = 0.0;
  __syncthreads();
  const int* mine_list = list + (int64_t)blockIdx.x * cap;
  const double* mine_w = wk + (int64_t)blockIdx.x * cap;
  const int nsel = __builtin_amdgcn_readfirstlane(cnt[blockIdx.x]);
  const int64_t nchunk = (nsel + BLOCK - 1) / BLOCK;
  for (int64_t it = 0; it < nchunk; ++it) {
    const int64_t j0 = it * BLOCK + tid;
    const bool live = j0 < nsel;
    const int64_t e = mine_list[live ? j0 : 0];
    double y[MAXD], x[MAXD];
    event_uniforms((uint64_t)e, iter, seed, 0, d, y);
    double jac = 1.0;
#pragma unroll
    for (int j = 0; j < MAXD; ++j)
      if (j < d) {
        int bin;
        x[j] = vegas_map_dim(edges + j * (nb + 1), nb, y[j], bin, jac);
      }
    const double thr = 4.0 * c.mt * c.mt, shat = x[0] * x[1] * c.s;
    V4<double> gl[NG > 0 ? NG : 1], top, atop;
    (void)phase_space<double>(NG, x, shat > thr ? shat : thr * (1.0 + 1e-3), c.mt, gl, top, atop);
    double v[N_OBS];
    v[0] = sqrt(top.x * top.x + top.y * top.y);
    const V4<double> P = top + atop;
    v[1] = sqrt(fmax(mdot(P, P), 0.0));
    v[2] = -1.0;
#pragma unroll
    for (int i = 0; i < NG; ++i) v[2] = fmax(v[2], sqrt(gl[i].x * gl[i].x + gl[i].y * gl[i].y));
    ws[tid] = live ? mine_w[j0] : 0.0;
#pragma unroll
    for (int q = 0; q < N_OBS; ++q) {
      const double t = (v[q] - o.lo[q]) * o.scale[q];
      ks[q * BLOCK + tid] = (live && t >= 0.0 && t < (double)onb) ? (int)t : -1;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < N_OBS) {
      double* h = hw + wave * W + lane * onb * 2;
      const int* kq = ks + lane * BLOCK + wave * 64;
      const double* wq = ws + wave * 64;
      for (int k = 0; k < 64; ++k) {
        const int b = kq[k];
        if (b >= 0) {
          h[2 * b] += wq[k];
          h[2 * b + 1] += wq[k] * wq[k];
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  __syncthreads();
  for (int i = tid; i < W; i += BLOCK) {
    double h = 0.0;
    for (int v2 = 0; v2 < WAVES; ++v2) h += hw[v2 * W + i];
    opart[(int64_t)blockIdx.x * W + i] = h;
  }
}

// ------------------------------------------------- gradient estimator
template <int NG, int CH, class RA>
__global__ void __launch_bounds__(BLOCK) k_grad_vegas(DevCfg c, const double* __restrict__ edges_g, uint64_t iter,
                                                      int64_t N, uint64_t seed, double* __restrict__ partials,
                                                      const int* __restrict__ list, const int* __restrict__ cnt,
                                                      int64_t cap) {
  extern __shared__ double lds[];
  const int d = c.ndim, nb = c.nb;
  const int tid = threadIdx.x, wave = tid >> 6;
  double* edges = lds;
  double* wacc = lds + d * (nb + 1);  // [WAVES][GV][4]: sum (hi, lo), sum of squares (hi, lo)
  for (int i = tid; i < d * (nb + 1); i += BLOCK) edges[i] = edges_g[i];
  for (int i = tid; i < WAVES * GV * 4; i += BLOCK) wacc[i] = 0.0;
  __syncthreads();
  double* acc = wacc + wave * GV * 4;
  // As in k_vegas, nothing per lane is carried across event chunks.
  // Only the events k_select kept: the others have zero weight and zero
  // pathwise derivatives (the cut boundaries do not move with the grid and
  // uniforms frozen).
  const int* mine_list = list + (int64_t)blockIdx.x * cap;
  const int nsel = __builtin_amdgcn_readfirstlane(cnt[blockIdx.x]);
  const int64_t nchunk = (nsel + BLOCK - 1) / BLOCK;
  for (int64_t it = 0; it < nchunk; ++it) {
    const int64_t j0 = it * BLOCK + tid;
    const bool live = j0 < nsel;
    const int64_t e = mine_list[live ? j0 : 0];
    double y[MAXD], x[MAXD];
    int bins[MAXD];
    event_uniforms((uint64_t)e, iter, seed, 0, d, y);
    double jac = 1.0;
#pragma unroll
    for (int j = 0; j < MAXD; ++j)
      if (j < d) x[j] = vegas_map_dim(edges + j * (nb + 1), nb, y[j], bins[j], jac);
    double v[GV];
    grad_event<NG, CH, RA>(c, x, v[0], v + 1);
    bool ok = live;
    for (int k = 0; k < GV; ++k) ok = ok && isfinite(v[k]);
    for (int k = 0; k < GV; ++k) {
      const double t = ok ? v[k] * jac : 0.0;
      double h, l;
      wave_sum_dd(t, h, l);
      lds_dd_accumulate(acc + 4 * k, h, l);
      wave_sum_dd(t * t, h, l);
      lds_dd_accumulate(acc + 4 * k + 2, h, l);
    }
  }
  __syncthreads();
  if (tid < GV) {
    const int k = tid;
    double hs = 0.0, ls = 0.0, hq = 0.0, lq = 0.0;
    for (int v = 0; v < WAVES; ++v) {
      const double* a = wacc + v * GV * 4 + 4 * k;
      dd_add(hs, ls, a[0]);
      dd_add(hs, ls, a[1]);
      dd_add(hq, lq, a[2]);
      dd_add(hq, lq, a[3]);
    }
    double* p = partials + (int64_t)blockIdx.x * (3 * GV);
    p[3 * k] = hs;
    p[3 * k + 1] = ls;
    p[3 * k + 2] = hq + lq;
  }
}

}  // namespace

// Launcher table of one (final gluons, channel, amplitude type) instance;
// GRAD = 0 leaves the derivative kernels out.
template <int NG, int CH, class RA, class RD, int GRAD, int FUSED = 1>
Launchers make_launchers() {
  Launchers L;
  L.fused = FUSED != 0;
  L.integrand = [](const DevCfg& c, const double* u, int64_t n, double* w, int nblk, int* list, int* cnt,
                   int64_t cap, hipStream_t s) {
    hipLaunchKernelGGL((k_select_points<NG>), dim3(nblk), dim3(BLOCK), 0, s, c, u, n, w, list, cnt, cap);
    hipLaunchKernelGGL((k_integrand<NG, CH, RA>), dim3(nblk), dim3(BLOCK), 0, s, c, u, n, w, list, cnt, cap);
  };
  L.vegas = [](const DevCfg& c, const double* edges, uint64_t iter, int64_t N, uint64_t seed, double* part,
               int pstride, int nblk, size_t lds, int* list, int* cnt, int64_t cap, double* wk, hipStream_t s) {
    hipLaunchKernelGGL((k_select<NG>), dim3(nblk), dim3(BLOCK), sizeof(double) * c.ndim * (c.nb + 1), s, c, edges,
                       iter, N, seed, list, cnt, cap);
    hipLaunchKernelGGL((k_vegas<NG, CH, RA>), dim3(nblk), dim3(BLOCK), lds, s, c, edges, iter, N, seed, part, pstride,
                       list, cnt, cap, wk);
  };
  L.observables = [](const DevCfg& c, const double* edges, uint64_t iter, uint64_t seed, const int* list,
                     const int* cnt, int64_t cap, const double* wk, const ObsSpec& o, double* opart, int nblk,
                     hipStream_t s) {
    const size_t lds = sizeof(double) * ((size_t)c.ndim * (c.nb + 1) + (size_t)WAVES * N_OBS * o.nbins * 2 + BLOCK) +
                       sizeof(int) * N_OBS * BLOCK;
    hipLaunchKernelGGL((k_observables<NG>), dim3(nblk), dim3(BLOCK), lds, s, c, edges, iter, seed, list, cnt, cap, wk,
                       o, opart);
  };
  L.integrand_grad = nullptr;
  L.grad_vegas = nullptr;
  L.integrand_ws = nullptr;
  L.ws_free = nullptr;
  if constexpr (GRAD != 0) {
    L.integrand_grad = [](const DevCfg& c, const double* u, int64_t n, double* w, double* dw, int nblk,
                          hipStream_t s) {
      hipLaunchKernelGGL((k_integrand_grad<NG, CH, RD>), dim3(nblk), dim3(BLOCK), 0, s, c, u, n, w, dw);
    };
    L.grad_vegas = [](const DevCfg& c, const double* edges, uint64_t iter, int64_t N, uint64_t seed, double* part,
                      int nblk, size_t lds, int* list, int* cnt, int64_t cap, hipStream_t s) {
      hipLaunchKernelGGL((k_select<NG>), dim3(nblk), dim3(BLOCK), sizeof(double) * c.ndim * (c.nb + 1), s, c, edges,
                         iter, N, seed, list, cnt, cap);
      hipLaunchKernelGGL((k_grad_vegas<NG, CH, RD>), dim3(nblk), dim3(BLOCK), lds, s, c, edges, iter, N, seed, part,
                         list, cnt, cap);
    };
  }
  return L;
}

}  // namespace mf
