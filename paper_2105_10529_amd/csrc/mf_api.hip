// Kernels and the C ABI of the per-event LO integrand library (gfx950).
//
// Kernels (one event per lane):
//   k_pdf_setup      tabulate the synthetic PDFs on the 196 x-knots and collapse
//                    the Q direction at the fixed scale (value, d/dmu, d/dtheta)
//   k_integrand      the integrand at caller-supplied points
//   k_integrand_grad the integrand and its forward-mode derivatives
//   k_vegas          one fused VEGAS iteration: Philox -> map -> phase space ->
//                    cuts -> PDFs -> |M|^2 -> weight -> compensated sums and
//                    per-wave grid histograms -> per-block partials
//   k_finalize       ordered reduction of the partials, iteration estimate,
//                    on-device grid refinement
//   k_refine         grid refinement alone
//   k_grad_vegas / k_grad_finalize   pathwise derivative estimates
// Sec. 2.1 of arXiv:2105.10529 describes the pipeline; Sec. 3.1 notes that
// everything stays in GPU memory, which is also the design here: one VEGAS
// iteration moves a few KB between host and device.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mf.h"
#include "../../include/mf_flow.h"
#include "flow_internal.h"
#include "launch.h"
#include "pipeline.h"
#include "status.h"

using namespace mf;

// Selection lists of mf_integrand_noalloc, in a device array of fixed size
// (never allocated at run time): [MAX_BLOCKS] per-block counts, then the
// per-block lists.  An n-point call with n <= NOALLOC_MAX_POINTS needs at most
// NOALLOC_MAX_POINTS list entries: below MAX_BLOCKS * BLOCK points the blocks
// hold one BLOCK-sized chunk each (ceil(n / BLOCK) * BLOCK entries), above it
// the MAX_BLOCKS blocks hold ceil(n / (MAX_BLOCKS * BLOCK)) chunks each, and
// NOALLOC_MAX_POINTS is a multiple of MAX_BLOCKS * BLOCK.  Each device keeps
// its own copy until the process ends; host code must use the address from
// hipGetSymbolAddress (g_noalloc_ptr), never the symbol itself.
constexpr int64_t NOALLOC_MAX_POINTS = MF_NOALLOC_MAX_POINTS;
static_assert(NOALLOC_MAX_POINTS % ((int64_t)MAX_BLOCKS * BLOCK) == 0, "list bound");
static __device__ __align__(256) int scratch[MAX_BLOCKS + NOALLOC_MAX_POINTS];


namespace mf {
namespace {
thread_local std::string g_err;
}
mf_status set_error(mf_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}
void clear_error() { mf::clear_error(); }
const char* last_error() { return g_err.c_str(); }
}  // namespace mf

namespace {

#define fail mf::set_error

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(MF_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr int RED_ROWS = 32;  // rows of the first reduction stage
constexpr int REC = 8;        // per-iteration record: I, sigma, S1, S2, nonzero, nonfinite, status, pad

struct PdfParams {
  double p[20];
};

// ------------------------------------------------------------ PDF tables
__device__ double pdf_formula(const double* p5, double x, double L, int dpar) {
  if (!(x < 1.0)) return 0.0;
  double lx = log(x), l1x = log1p(-x);
  double v = p5[0] * exp((p5[1] + p5[2] * L) * lx + (p5[3] + p5[4] * L) * l1x);
  switch (dpar) {
    case 0: return v / p5[0];
    case 1: return v * lx;
    case 2: return v * L * lx;
    case 3: return v * l1x;
    case 4: return v * L * l1x;
    default: return v;
  }
}

// One thread per (flavour, x knot): Hermite in ln Q at mu of the tabulated
// values (and of the parameter derivatives), with its mu derivative.
__global__ void k_pdf_setup(PdfParams P, double mu, double* pdfc, double* pdfd, double* pdft) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * NXK) return;
  int f = t / NXK, i = t % NXK;
  double x = pow(10.0, -9.0 + 9.0 * i / 195.0);
  double hq = (log(PDF_QMAX) - log(PDF_Q0)) / (NQK - 1);
  double tq = (log(mu) - log(PDF_Q0)) / hq;
  int j = (int)floor(tq);
  j = j < 0 ? 0 : (j > NQK - 2 ? NQK - 2 : j);
  double u = tq - j;
  double u2 = u * u, u3 = u2 * u;
  double h00 = 2 * u3 - 3 * u2 + 1, h10 = u3 - 2 * u2 + u, h01 = -2 * u3 + 3 * u2, h11 = u3 - u2;
  double d00 = 6 * u2 - 6 * u, d10 = 3 * u2 - 4 * u + 1, d01 = -6 * u2 + 6 * u, d11 = 3 * u2 - 2 * u;
  // theta_k -> (flavour, parameter): A_g a_g b_g c_g d_g A_u A_d A_u~
  const int tf[8] = {0, 0, 0, 0, 0, 1, 2, 3}, tp[8] = {0, 1, 2, 3, 4, 0, 0, 0};
  for (int which = -1; which < 8; ++which) {
    if (which >= 0 && tf[which] != f) continue;
    int dpar = which < 0 ? -1 : tp[which];
    double F[4];
    for (int r = 0; r < 4; ++r) {
      int jj = j - 1 + r;
      jj = jj < 0 ? 0 : (jj > NQK - 1 ? NQK - 1 : jj);
      double Q = PDF_Q0 * pow(PDF_QMAX / PDF_Q0, jj / 49.0);
      F[r] = pdf_formula(P.p + 5 * f, x, log(Q / PDF_Q0), dpar);
    }
    // F[1] = row j, F[2] = row j+1
    double s0 = (j == 0) ? F[2] - F[1] : 0.5 * (F[2] - F[0]);
    double s1 = (j + 1 == NQK - 1) ? F[2] - F[1] : 0.5 * (F[3] - F[1]);
    double v = h00 * F[1] + h10 * s0 + h01 * F[2] + h11 * s1;
    if (which < 0) {
      pdfc[f * NXK + i] = v;
      pdfd[f * NXK + i] = (d00 * F[1] + d10 * s0 + d01 * F[2] + d11 * s1) / (hq * mu);
    } else {
      pdft[which * NXK + i] = v;
    }
  }
}

// The full knot table x f(x_i, Q_j) of the four flavours, [4][50][196], for
// the dynamic scale (the same knots and formula as the fixed-scale set-up).
__global__ void k_pdf_table(PdfParams P, double* tab) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4 * NQK * NXK) return;
  const int f = t / (NQK * NXK), j = (t / NXK) % NQK, i = t % NXK;
  const double x = pow(10.0, -9.0 + 9.0 * i / 195.0);
  const double Q = PDF_Q0 * pow(PDF_QMAX / PDF_Q0, j / 49.0);
  tab[t] = pdf_formula(P.p + 5 * f, x, log(Q / PDF_Q0), -1);
}

__global__ void k_fill_uniform(double* edges, int d, int nb) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d * (nb + 1)) return;
  int k = t % (nb + 1);
  edges[t] = (double)k / nb;
}

// ------------------------------------------------------- staged iteration
// Points kernel: Philox uniforms through the grid; writes the mapped point
// [ndim][N], the Jacobian [N] and the bin indices [ndim][N].
__global__ void __launch_bounds__(256) k_stage_points(const double* __restrict__ edges_g, int d, int nb, uint64_t iter,
                                                      int64_t N, uint64_t seed, double* __restrict__ x,
                                                      double* __restrict__ jac, unsigned char* __restrict__ bins) {
  extern __shared__ double edges[];
  for (int i = threadIdx.x; i < d * (nb + 1); i += blockDim.x) edges[i] = edges_g[i];
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * blockDim.x, stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t nchunk = b0 < N ? (N - b0 + stride - 1) / stride : 0;
  for (int64_t it = 0; it < nchunk; ++it) {
    const int64_t e = b0 + it * stride + threadIdx.x;
    if (e >= N) continue;
    double y[MAXD];
    event_uniforms((uint64_t)e, iter, seed, 0, d, y);
    double J = 1.0;
    for (int j = 0; j < d; ++j) {
      int b;
      x[(int64_t)j * N + e] = vegas_map_dim(edges + j * (nb + 1), nb, y[j], b, J);
      bins[(int64_t)j * N + e] = (unsigned char)b;
    }
    jac[e] = J;
  }
}

// Points of a frozen-grid sample: y from Philox (yin == NULL, key word 1 =
// purpose) or from the caller (FP32, e.g. drawn by the flow); x = map(y), the
// Jacobian (divided by a + (1 - a) exp(logq) when logq is given: the weight
// of a point drawn from that density in y), bins, and optionally y as FP32.
__global__ void __launch_bounds__(256) k_sample_points(const double* __restrict__ edges_g, int d, int nb, uint64_t iter,
                                                       int64_t N, uint64_t seed, uint64_t purpose,
                                                       const float* __restrict__ yin, const float* __restrict__ logq,
                                                       double mix, float* __restrict__ yout, double* __restrict__ x,
                                                       double* __restrict__ jac, unsigned char* __restrict__ bins) {
  extern __shared__ double edges[];
  for (int i = threadIdx.x; i < d * (nb + 1); i += blockDim.x) edges[i] = edges_g[i];
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * blockDim.x, stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t nchunk = b0 < N ? (N - b0 + stride - 1) / stride : 0;
  for (int64_t it = 0; it < nchunk; ++it) {
    const int64_t e = b0 + it * stride + threadIdx.x;
    if (e >= N) continue;
    double y[MAXD];
    if (yin) {
      for (int j = 0; j < d; ++j) y[j] = (double)yin[(int64_t)j * N + e];
    } else {
      event_uniforms((uint64_t)e, iter, seed, purpose, d, y);
    }
    double J = 1.0;
    for (int j = 0; j < d; ++j) {
      int b;
      x[(int64_t)j * N + e] = vegas_map_dim(edges + j * (nb + 1), nb, y[j], b, J);
      bins[(int64_t)j * N + e] = (unsigned char)b;
      if (yout) yout[(int64_t)j * N + e] = (float)y[j];
    }
    if (logq) J /= mix + (1.0 - mix) * exp((double)logq[e]);
    jac[e] = J;
  }
}

// FP32 Philox uniforms [d][N] (key (seed, purpose), counter (e, iter, call, 0)).
__global__ void __launch_bounds__(256) k_uniform_f32(int d, uint64_t iter, int64_t N, uint64_t seed, uint64_t purpose,
                                                     float* __restrict__ out) {
  const int64_t b0 = (int64_t)blockIdx.x * blockDim.x, stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t nchunk = b0 < N ? (N - b0 + stride - 1) / stride : 0;
  for (int64_t it = 0; it < nchunk; ++it) {
    const int64_t e = b0 + it * stride + threadIdx.x;
    if (e >= N) continue;
    double u[MAXD];
    event_uniforms((uint64_t)e, iter, seed, purpose, d, u);
    for (int j = 0; j < d; ++j) out[(int64_t)j * N + e] = (float)u[j];
  }
}

// w[e] = f[e] * jac[e] (non-finite products give 0)
__global__ void k_weight(const double* __restrict__ f, const double* __restrict__ jac, int64_t N,
                         double* __restrict__ w) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  const double v = f[e] * jac[e];
  w[e] = isfinite(v) ? v : 0.0;
}

// Per-sample weights of an on-policy training step from points drawn from
// the mixture q_m = a + (1 - a) q: with r = f J / q_m (the sample weight),
// the gradient of int p^2 / q_m is -(1-a) E_qm[r^2 (q/q_m) grad log q] and
// that of the forward KL is -(1-a) E_qm[r (q/q_m) grad log q]; out[e] is
// r^2 q/q_m (variance) or r q/q_m (KL) in FP32, and r2[e] = r^2 for the
// batch's relative-variance estimate.
__global__ void k_online_weights(const double* __restrict__ f, const double* __restrict__ jac,
                                 const float* __restrict__ logq, double mix, int64_t N, int variance,
                                 float* __restrict__ out, float* __restrict__ rw, float* __restrict__ r2,
                                 int* __restrict__ bad) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  double r = f[e] * jac[e];
  // a non-finite density or Jacobian means the proposal itself is broken (a
  // diverged training step): flagged, so the caller can stop instead of
  // silently dropping those points from the estimate
  if (!isfinite(r) || !isfinite(logq[e])) *bad = 1;
  r = isfinite(r) ? r : 0.0;
  const double q = exp((double)logq[e]);
  const double share = q / (mix + (1.0 - mix) * q);
  out[e] = (float)((variance ? r * r : r) * share);
  rw[e] = (float)r;
  r2[e] = (float)(r * r);
}

// relative variance per event of a batch of sample weights r,
// n sum r^2 / (sum r)^2 - 1, and the sums (sum r, sum r^2) in FP64
__global__ void __launch_bounds__(1024) k_batch_relvar(const float* __restrict__ r, const float* __restrict__ r2,
                                                       int64_t n, float* __restrict__ out, double* __restrict__ sums) {
  __shared__ double s1[1024], s2[1024];
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    a += r[i];
    b += r2[i];
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int st = 512; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      s1[threadIdx.x] += s1[threadIdx.x + st];
      s2[threadIdx.x] += s2[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = (float)((double)n * s2[0] / (s1[0] * s1[0]) - 1.0);
    sums[0] = s1[0];
    sums[1] = s2[0];
  }
}

// Accumulation kernel: weights w*J into the same per-block partials as the
// fused kernel (compensated sums from deterministic wave reductions, per-wave
// histograms combined in order).
__global__ void __launch_bounds__(256) k_stage_accumulate(const double* __restrict__ f, const double* __restrict__ jac,
                                                          const unsigned char* __restrict__ bins, int d, int nb,
                                                          int64_t N, double* __restrict__ partials, int pstride) {
  __shared__ double hist[WAVES][MAXD * MAX_BINS];
  __shared__ double wacc[WAVES][4];
  __shared__ unsigned long long cnt[2 * WAVES];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = lane; i < d * nb; i += 64) hist[wave][i] = 0.0;
  if (lane < 4) wacc[wave][lane] = 0.0;
  __syncthreads();
  unsigned long long nnz = 0, nbad = 0;
  const int64_t b0 = (int64_t)blockIdx.x * BLOCK, stride = (int64_t)gridDim.x * BLOCK;
  const int64_t nchunk = b0 < N ? (N - b0 + stride - 1) / stride : 0;
  for (int64_t it = 0; it < nchunk; ++it) {
    const int64_t e0 = b0 + it * stride + tid;
    const bool live = e0 < N;
    const int64_t e = live ? e0 : N - 1;
    double w = f[e] * jac[e];
    const bool finite = isfinite(w);
    nbad += __popcll(__ballot(live && !finite));
    w = (live && finite) ? w : 0.0;
    nnz += __popcll(__ballot(w != 0.0));
    double h, l;
    wave_sum_dd(w, h, l);
    lds_dd_accumulate(wacc[wave], h, l);
    wave_sum_dd(w * w, h, l);
    lds_dd_accumulate(wacc[wave] + 2, h, l);
    // bin in event order: lane j < d walks the wave's 64 events of dimension j
    const double w2 = w * w;
    for (int k = 0; k < 64; ++k) {
      const double wk = __shfl(w2, k);
      const int64_t ek = __shfl(e, k);
      if (lane < d) hist[wave][lane * nb + bins[(int64_t)lane * N + ek]] += wk;
    }
  }
  __syncthreads();
  double* p = partials + (int64_t)blockIdx.x * pstride;
  for (int i = tid; i < d * nb; i += BLOCK) {
    double s = 0.0;
    for (int v = 0; v < WAVES; ++v) s += hist[v][i];
    p[PART_HEAD + i] = s;
  }
  if (lane == 0) {
    cnt[wave] = nnz;
    cnt[WAVES + wave] = nbad;
  }
  __syncthreads();
  if (tid == 0) {
    double h1 = 0.0, l1 = 0.0, h2 = 0.0, l2 = 0.0;
    unsigned long long tn = 0, tb = 0;
    for (int v = 0; v < WAVES; ++v) {
      dd_add(h1, l1, wacc[v][0]);
      dd_add(h1, l1, wacc[v][1]);
      dd_add(h2, l2, wacc[v][2]);
      dd_add(h2, l2, wacc[v][3]);
      tn += cnt[v];
      tb += cnt[WAVES + v];
    }
    p[0] = h1;
    p[1] = l1;
    p[2] = h2;
    p[3] = l2;
    p[4] = (double)tn;
    p[5] = (double)tb;
  }
}

// -------------------------------------------------------- refinement
// Lepage's refinement of one dimension, serial over bins (50-ish), FP64.
// Returns false (and leaves e unchanged) if the new edges are not strictly
// increasing.
__device__ bool refine_dim(double* e, const double* h, int nb, double alpha, double* scratch) {
  double* dsm = scratch;       // nb
  double* r = scratch + nb;    // nb
  double* ne = scratch + 2 * nb;  // nb+1
  if (nb == 1) dsm[0] = h[0];
  else {
    dsm[0] = 0.5 * (h[0] + h[1]);
    dsm[nb - 1] = 0.5 * (h[nb - 2] + h[nb - 1]);
    for (int k = 1; k < nb - 1; ++k) dsm[k] = (h[k - 1] + h[k] + h[k + 1]) / 3.0;
  }
  double D = 0.0;
  for (int k = 0; k < nb; ++k) D += dsm[k];
  if (!(D > 0.0)) return true;
  double Rs = 0.0;
  for (int k = 0; k < nb; ++k) {
    double rk = 0.0;
    if (dsm[k] > 0.0) {
      double q = dsm[k] / D;
      rk = (q < 1.0) ? pow((1.0 - q) / log(1.0 / q), alpha) : 0.0;
    }
    r[k] = rk;
    Rs += rk;
  }
  if (!(Rs > 0.0)) return true;
  double per = Rs / nb;
  ne[0] = e[0];
  ne[nb] = e[nb];
  int k = 0;
  double acc = 0.0;
  for (int i = 1; i < nb; ++i) {
    double target = per * i;
    while (k < nb && acc + r[k] < target) {
      acc += r[k];
      ++k;
    }
    ne[i] = (k >= nb) ? e[nb] : e[k] + (target - acc) / r[k] * (e[k + 1] - e[k]);
  }
  for (int i = 0; i < nb; ++i)
    if (!(ne[i + 1] > ne[i])) return false;
  for (int i = 0; i <= nb; ++i) e[i] = ne[i];
  return true;
}

__global__ void k_clear_status(int* status) { status[0] = 0; }

__global__ void k_refine(double* edges, const double* hist, int d, int nb, double alpha, int* status) {
  __shared__ double scratch[3 * MAX_BINS + 1];
  int j = blockIdx.x;
  if (threadIdx.x == 0 && j < d) {
    bool ok = refine_dim(edges + j * (nb + 1), hist + j * nb, nb, alpha, scratch);
    if (!ok) status[0] = 1;
  }
}

// First reduction stage: block r of R sums the partials of source blocks
// [r*nblk/R, (r+1)*nblk/R) in order and writes one row in the same layout
// (compensated pairs stay pairs).  A fixed partition keeps the result
// bitwise reproducible; R rows then go to the single-block finaliser.
__global__ void k_reduce_partials(const double* partials, int nblk, int pstride, int width, int R, double* out) {
  const int r = blockIdx.x;
  const int b0 = (int)((int64_t)r * nblk / R), b1 = (int)((int64_t)(r + 1) * nblk / R);
  double* o = out + (int64_t)r * pstride;
  for (int i = threadIdx.x; i < width; i += blockDim.x) {
    if (i == 1 || i == 3) continue;  // low words are folded into their pair below
    if (i == 0 || i == 2) {
      double hi = 0.0, lo = 0.0;
      for (int b = b0; b < b1; ++b) {
        dd_add(hi, lo, partials[(int64_t)b * pstride + i]);
        dd_add(hi, lo, partials[(int64_t)b * pstride + i + 1]);
      }
      o[i] = hi;
      o[i + 1] = lo;
    } else {
      double acc = 0.0;
      for (int b = b0; b < b1; ++b) acc += partials[(int64_t)b * pstride + i];
      o[i] = acc;
    }
  }
}

// Column sums of the observables' block partial rows [nblk][W] in a fixed
// order: stage 1 sums row groups (grid (ceil(W/256), R)), stage 2 adds the R
// group sums, in order, to the running histogram.
__global__ void k_obs_reduce(const double* part, int nblk, int W, int R, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  if (i >= W) return;
  const int b0 = (int)((int64_t)r * nblk / R), b1 = (int)((int64_t)(r + 1) * nblk / R);
  double acc = 0.0;
  for (int b = b0; b < b1; ++b) acc += part[(int64_t)b * W + i];
  out[(int64_t)r * W + i] = acc;
}
__global__ void k_obs_accumulate(const double* rows, int R, int W, double* sums) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= W) return;
  double acc = 0.0;
  for (int r = 0; r < R; ++r) acc += rows[(int64_t)r * W + i];
  sums[i] += acc;
}

// Ordered reduction of the block partials of one iteration; writes the
// iteration record and (if adapt) refines the grid in place.
__global__ void k_finalize(const double* partials, int nblk, int pstride, int d, int nb, int64_t N, double alpha,
                           int adapt, double* edges, double* rec, double* hist_out) {
  __shared__ double hsum[MAXD * MAX_BINS];
  __shared__ double scratch[MAXD][3 * MAX_BINS + 1];
  const int tid = threadIdx.x;
  for (int i = tid; i < d * nb; i += blockDim.x) {
    double h = 0.0;
    for (int b = 0; b < nblk; ++b) h += partials[(int64_t)b * pstride + PART_HEAD + i];
    hsum[i] = h;
    if (hist_out) hist_out[i] = h;
  }
  __syncthreads();
  if (tid == 0) {
    double h1 = 0.0, l1 = 0.0, h2 = 0.0, l2 = 0.0, nz = 0.0, bad = 0.0;
    for (int b = 0; b < nblk; ++b) {
      const double* p = partials + (int64_t)b * pstride;
      dd_add(h1, l1, p[0]);
      dd_add(h1, l1, p[1]);
      dd_add(h2, l2, p[2]);
      dd_add(h2, l2, p[3]);
      nz += p[4];
      bad += p[5];
    }
    double S1 = h1 + l1, S2 = h2 + l2;
    double I = S1 / (double)N;
    double var = (S2 / (double)N - I * I) / (double)(N - 1);
    rec[0] = I;
    rec[1] = sqrt(var > 0.0 ? var : 0.0);
    rec[2] = S1;
    rec[3] = S2;
    rec[4] = nz;
    rec[5] = bad;
    rec[6] = 0.0;
  }
  __syncthreads();
  if (adapt && tid < d) {
    bool ok = refine_dim(edges + tid * (nb + 1), hsum + tid * nb, nb, alpha, scratch[tid]);
    if (!ok) rec[6] = 1.0;
  }
}

__global__ void k_grad_finalize(const double* partials, int nblk, int64_t N, double* out) {
  int k = threadIdx.x;
  if (k >= GV) return;
  double hi = 0.0, lo = 0.0, q = 0.0;
  for (int b = 0; b < nblk; ++b) {
    dd_add(hi, lo, partials[(int64_t)b * 3 * GV + 3 * k]);
    dd_add(hi, lo, partials[(int64_t)b * 3 * GV + 3 * k + 1]);
    q += partials[(int64_t)b * 3 * GV + 3 * k + 2];
  }
  double mean = (hi + lo) / (double)N;
  double var = (q / (double)N - mean * mean) / (double)(N - 1);
  out[k] = mean;
  out[GV + k] = sqrt(var > 0.0 ? var : 0.0);
}

}  // namespace

// ============================================================== host side
struct mf_process {
  mf_config cfg;
  DevCfg dc;
  int device;
  int ndim, nb;
  double* d_pdf = nullptr;      // pdfc | pdfd | pdft
  double* d_edges = nullptr;    // ndim*(nb+1)
  double* d_part = nullptr;     // MAX_BLOCKS * pstride
  double* d_part2 = nullptr;    // RED_ROWS * pstride (first reduction stage)
  double* d_rec = nullptr;      // per-iteration records
  double* d_hist = nullptr;     // last histogram
  double* d_out = nullptr;      // small outputs
  int* d_status = nullptr;
  int pstride;
  int rec_cap;
  Launchers L;
  // staged-iteration buffers (allocated on first use, grown on demand)
  int64_t stage_cap = 0;
  double* d_sx = nullptr;          // [ndim][cap]
  double* d_sjac = nullptr;        // [cap]
  double* d_sw = nullptr;          // [cap]
  unsigned char* d_sbins = nullptr;  // [ndim][cap]
  float* d_sy = nullptr;           // [ndim][cap] flow points (FP32)
  float* d_slq = nullptr;          // [cap] flow log-density
  float* d_sz = nullptr;           // [ndim][cap] scratch for the flow's density pass
  float* d_sw32 = nullptr;         // [3][cap] on-policy training weights
  void* ws = nullptr;              // workspace of a multi-kernel integrand (Launchers::integrand_ws)
  // per-block lists of the events that pass the cuts (fused iterations)
  int64_t sel_cap = 0;             // list entries per block
  int* d_sel = nullptr;            // [MAX_BLOCKS][sel_cap]
  int* d_selcnt = nullptr;         // [MAX_BLOCKS]
  double* d_selw = nullptr;        // [MAX_BLOCKS][sel_cap] weights of the kept events (observables)
  int64_t selw_cap = 0;
  double* d_obs = nullptr;         // observables: block partials, reduced rows, running sums
  double* d_pdfq = nullptr;        // [4][50][196] full PDF knot table (dynamic scale)
};

namespace {

// Massless final-state partons (gluons, or the light quark of q g -> t t~ q).
int n_final_gluons(int proc) {
  switch (proc) {
    case MF_GG_TTXG:
    case MF_UUX_TTXG:
    case MF_DDX_TTXG:
    case MF_QG_TTXQ: return 1;
    case MF_GG_TTXGG: return 2;
    case MF_GG_TTXGGG: return 3;
    default: return 0;
  }
}
// 0: g g; 1: u u~; 2: d d~; 3: q g (q = u, d, u~, d~)
int channel_of(int proc) {
  switch (proc) {
    case MF_UUX_TTX:
    case MF_UUX_TTXG: return 1;
    case MF_DDX_TTX:
    case MF_DDX_TTXG: return 2;
    case MF_QG_TTXQ: return 3;
    default: return 0;
  }
}

double factorial(int n) {
  double f = 1;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

int blocks_for(int64_t n) {
  int64_t b = (n + BLOCK - 1) / BLOCK;
  if (b < 1) b = 1;
  if (b > MAX_BLOCKS) b = MAX_BLOCKS;
  return (int)b;
}

// Blocks of a VEGAS iteration: once there are more than 256 chunks of
// events, at least 16 chunks per block, in whole rounds of 256 blocks (the
// fused kernel runs one block per compute unit at a time), so that a
// block's kept events fill several passes of its waves and no round is
// mostly idle; one chunk per block up to 256 chunks.
int iter_blocks(int64_t n) {
  const int64_t chunks = (n + BLOCK - 1) / BLOCK;
  if (chunks <= 256) return blocks_for(n);
  int64_t b = (chunks + 15) / 16;
  b = (b + 255) / 256 * 256;
  if (b < 256) b = 256;
  if (b > MAX_BLOCKS) b = MAX_BLOCKS;
  return (int)b;
}

size_t vegas_lds_bytes(int d, int nb) {
  return sizeof(double) * (size_t)(d * (nb + 1) + 4 * NXK + WAVES * (d + 1) * nb + WAVES * 4 + 2 * BLOCK +
                                  d * BLOCK) +
         (size_t)d * BLOCK;
}

// Colour form of g g -> t t~ g g when the configuration leaves it open: the
// in-register form, measured faster in both precisions (FP32: 1.07e8 against
// 0.89e8 events/s; FP64: 7.3e7 against 3.6e7).
int default_colour_form(int) { return 1; }

Launchers pick_launchers(int ng, int ch, int prec, int colour_form) {
  const bool f32 = prec == MF_PREC_FP32_AMP;
  if (ch == 1) return ng == 1 ? launchers_uug_f64() : launchers_uu_f64();
  if (ch == 2) return ng == 1 ? launchers_ddg_f64() : launchers_dd_f64();
  if (ch == 3) return launchers_qg_f64();
  if (ng == 0) return f32 ? launchers_gg0_f32() : launchers_gg0_f64();
  if (ng == 1) return f32 ? launchers_gg1_f32() : launchers_gg1_f64();
  if (ng == 3) return f32 ? launchers_gg3_f32() : launchers_gg3_f64();
  if (colour_form == 2) return f32 ? launchers_gg2s_f32() : launchers_gg2s_f64();
  return f32 ? launchers_gg2_f32() : launchers_gg2_f64();
}

mf_status check_stream_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(MF_EDEVICE, "%s launch: %s", what, hipGetErrorString(e));
  return MF_OK;
}

constexpr int MAX_DEVICES = 64;
std::mutex g_noalloc_mtx;
int* g_noalloc_ptr[MAX_DEVICES] = {};
hipError_t g_noalloc_err[MAX_DEVICES] = {};

// Look up this device's copy of the scratch array once, with the device current.
void noalloc_scratch_init(int dev) {
  if (dev < 0 || dev >= MAX_DEVICES) return;
  std::lock_guard<std::mutex> lock(g_noalloc_mtx);
  if (g_noalloc_ptr[dev]) return;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  g_noalloc_err[dev] = e;
  if (e == hipSuccess) g_noalloc_ptr[dev] = static_cast<int*>(ptr);
  else (void)hipGetLastError();
}

// Grow the per-block selection lists to the chunks of an n-event pass over
// nblk blocks.
mf_status ensure_select(mf_process* p, int64_t n, int nblk, hipStream_t s) {
  if (n > (int64_t)INT32_MAX) return fail(MF_EINVAL, "n_events must be below 2^31 for fused iterations");
  const int64_t cap = (n + (int64_t)nblk * BLOCK - 1) / ((int64_t)nblk * BLOCK) * BLOCK;
  if (p->d_selcnt && p->sel_cap >= cap) return MF_OK;
  HIP_TRY(hipStreamSynchronize(s));
  (void)hipFree(p->d_sel);
  p->d_sel = nullptr;
  p->sel_cap = 0;
  if (!p->d_selcnt && hipMalloc(&p->d_selcnt, sizeof(int) * MAX_BLOCKS) != hipSuccess)
    return fail(MF_ENOMEM, "selection counts");
  if (hipMalloc(&p->d_sel, sizeof(int) * (size_t)MAX_BLOCKS * cap) != hipSuccess)
    return fail(MF_ENOMEM, "selection lists (%lld events)", (long long)n);
  p->sel_cap = cap;
  return MF_OK;
}

// The integrand of the process on n mapped points (single-kernel or staged).
mf_status run_integrand(mf_process* p, const double* x, int64_t n, double* w, hipStream_t s) {
  if (p->L.integrand_ws) {
    hipError_t e = p->L.integrand_ws(p->dc, x, n, w, &p->ws, s);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
      return fail(MF_ENOMEM, "integrand workspace allocation failed");
    if (e != hipSuccess) return fail(MF_EDEVICE, "integrand: %s", hipGetErrorString(e));
    return MF_OK;
  }
  mf_status st = ensure_select(p, n, blocks_for(n), s);
  if (st != MF_OK) return st;
  p->L.integrand(p->dc, x, n, w, blocks_for(n), p->d_sel, p->d_selcnt, p->sel_cap, s);
  return check_stream_launch("k_integrand");
}

// Grow the staging buffers of the handle to n events.
mf_status ensure_stage(mf_process* p, int64_t n, hipStream_t s) {
  if (p->stage_cap >= n) return MF_OK;
  HIP_TRY(hipStreamSynchronize(s));
  hipFree(p->d_sx);
  hipFree(p->d_sjac);
  hipFree(p->d_sw);
  hipFree(p->d_sbins);
  hipFree(p->d_sy);
  hipFree(p->d_slq);
  hipFree(p->d_sz);
  hipFree(p->d_sw32);
  p->d_sx = p->d_sjac = p->d_sw = nullptr;
  p->d_sbins = nullptr;
  p->d_sy = p->d_slq = p->d_sz = p->d_sw32 = nullptr;
  p->stage_cap = 0;
  const size_t d = (size_t)p->ndim, m = (size_t)n;
  if (hipMalloc(&p->d_sx, sizeof(double) * d * m) != hipSuccess || hipMalloc(&p->d_sjac, sizeof(double) * m) != hipSuccess ||
      hipMalloc(&p->d_sw, sizeof(double) * m) != hipSuccess || hipMalloc(&p->d_sbins, d * m) != hipSuccess ||
      hipMalloc(&p->d_sy, sizeof(float) * d * m) != hipSuccess || hipMalloc(&p->d_slq, sizeof(float) * m) != hipSuccess ||
      hipMalloc(&p->d_sz, sizeof(float) * d * m) != hipSuccess ||
      hipMalloc(&p->d_sw32, sizeof(float) * 3 * m) != hipSuccess) {
    hipGetLastError();
    return fail(MF_ENOMEM, "staging buffers for %lld events", (long long)n);
  }
  p->stage_cap = n;
  return MF_OK;
}

// Points and Jacobians of one frozen-grid sample into the staging buffers.
// VEGAS: Philox y -> map.  Flow with mixture fraction a: Philox numbers with
// key word 1; events e < floor(a n) use them as y directly (their flow
// density from a density pass on a copy), the others as z through the
// flow's sampling direction; every weight is divided by a + (1 - a) q(y).
mf_status stage_sample(mf_process* p, mf_flow* flow, double mix, uint64_t iter, int64_t n, float* yout,
                       hipStream_t s) {
  const int d = p->ndim, nb = p->nb;
  const int nblk = blocks_for(n);
  const size_t lds = sizeof(double) * d * (nb + 1);
  if (flow) {
    hipLaunchKernelGGL(k_uniform_f32, dim3(nblk), dim3(256), 0, s, d, iter, n, p->cfg.seed, (uint64_t)1, p->d_sy);
    const int64_t nu = (int64_t)std::floor(mix * (double)n);
    mf_status st = mf::flow_apply(flow, p->d_sy + nu, n - nu, n, p->d_slq + nu, true, s);
    if (st != MF_OK) return st;
    if (nu > 0) {
      HIP_TRY(hipMemcpy2DAsync(p->d_sz, sizeof(float) * nu, p->d_sy, sizeof(float) * n, sizeof(float) * nu, d,
                               hipMemcpyDeviceToDevice, s));
      st = mf::flow_apply(flow, p->d_sz, nu, nu, p->d_slq, false, s);
      if (st != MF_OK) return st;
    }
    hipLaunchKernelGGL(k_sample_points, dim3(nblk), dim3(256), lds, s, p->d_edges, d, nb, iter, n, p->cfg.seed,
                       (uint64_t)1, p->d_sy, p->d_slq, mix, yout, p->d_sx, p->d_sjac, p->d_sbins);
  } else {
    hipLaunchKernelGGL(k_sample_points, dim3(nblk), dim3(256), lds, s, p->d_edges, d, nb, iter, n, p->cfg.seed,
                       (uint64_t)0, (const float*)nullptr, (const float*)nullptr, 0.0, yout, p->d_sx, p->d_sjac,
                       p->d_sbins);
  }
  return check_stream_launch("k_sample_points");
}


}  // namespace

extern "C" {

const char* mf_last_error(void) { return mf::last_error(); }

int mf_process_ndim(const mf_process* p) { return p ? p->ndim : 0; }

mf_status mf_process_create(const mf_config* cfg, mf_process** out) {
  mf::clear_error();
  if (!cfg || !out) return fail(MF_EINVAL, "NULL argument");
  *out = nullptr;
  if (cfg->process < MF_GG_TTX || cfg->process > MF_QG_TTXQ) return fail(MF_EINVAL, "unknown process %d", cfg->process);
  if (cfg->precision != MF_PREC_FP64 && cfg->precision != MF_PREC_FP32_AMP)
    return fail(MF_EINVAL, "unknown precision %d", cfg->precision);
  if (!(cfg->m_t > 0.0)) return fail(MF_EINVAL, "m_t must be positive");
  if (!(cfg->sqrt_s > 2.0 * cfg->m_t)) return fail(MF_EINVAL, "sqrt_s must exceed 2 m_t");
  if (!(cfg->alpha_s > 0.0)) return fail(MF_EINVAL, "alpha_s must be positive");
  if (!(cfg->alpha > 0.0)) return fail(MF_EINVAL, "VEGAS alpha must be positive");
  if (cfg->n_bins < 1 || cfg->n_bins > MAX_BINS) return fail(MF_EINVAL, "n_bins must be in 1..%d", MAX_BINS);
  double mu = cfg->mu > 0.0 ? cfg->mu : cfg->m_t;
  if (!(mu >= PDF_Q0 && mu <= PDF_QMAX)) return fail(MF_ERANGE, "scale %g outside the PDF grid", mu);
  const int ng = n_final_gluons(cfg->process);
  if (cfg->helicity < 0 || cfg->helicity > 2 + 63) return fail(MF_EINVAL, "helicity mode %d", cfg->helicity);
  if (cfg->helicity != 0 && ng != 3)
    return fail(MF_ENOTSUP, "polarisation-state sampling is built for g g -> t t~ g g g only");
  if (cfg->dynamic_scale != 0 && cfg->dynamic_scale != 1)
    return fail(MF_EINVAL, "dynamic_scale must be 0 or 1");
  if (cfg->colour_form < 0 || cfg->colour_form > 2) return fail(MF_EINVAL, "colour_form must be 0, 1 or 2");
  if (cfg->colour_form != 0 && ng != 2)
    return fail(MF_ENOTSUP, "the colour form is selectable for g g -> t t~ g g only");
  if (channel_of(cfg->process) != 0 && cfg->precision != MF_PREC_FP64)
    return fail(MF_ENOTSUP, "quark channels are built in FP64 only");
  for (int i = 0; i < 20; i += 5)
    if (!(cfg->pdf_params[i] > 0.0)) return fail(MF_EINVAL, "PDF normalisation %d must be positive", i / 5);

  mf_process* p = new mf_process();
  p->cfg = *cfg;
  hipGetDevice(&p->device);
  noalloc_scratch_init(p->device);
  p->ndim = 3 * (ng + 2) - 2;
  p->nb = cfg->n_bins;
  DevCfg& c = p->dc;
  c.ng = ng;
  c.channel = channel_of(cfg->process);
  c.ndim = p->ndim;
  c.nb = p->nb;
  c.s = cfg->sqrt_s * cfg->sqrt_s;
  c.mt = cfg->m_t;
  c.mu = mu;
  c.mu_is_mt = cfg->mu > 0.0 ? 0 : 1;
  c.helicity = cfg->helicity;
  c.seed = cfg->seed;
  c.dyn_scale = cfg->dynamic_scale;
  c.pdfq = nullptr;
  c.pt_min = cfg->pt_min;
  c.eta_max = cfg->eta_max;
  c.dr_min = cfg->dr_min;
  c.lx0 = std::log(std::pow(10.0, -9.0));
  c.ihx = (NXK - 1) / (0.0 - c.lx0);
  double g2 = 4.0 * M_PI * cfg->alpha_s;
  // coupling g^(2 n), initial spin and colour average, final-state symmetry
  if (c.channel == 0) c.norm = std::pow(g2, ng + 2) / 256.0 / factorial(ng) * GEV2_PB;
  else if (c.channel == 3) c.norm = g2 * g2 * g2 / 96.0 * GEV2_PB;
  else c.norm = std::pow(g2, ng + 2) / 36.0 * GEV2_PB;
  const int colour_form = cfg->colour_form != 0 ? cfg->colour_form : default_colour_form(cfg->precision);
  p->L = pick_launchers(ng, c.channel, cfg->precision, ng == 2 ? colour_form : 1);
  p->pstride = PART_HEAD + p->ndim * p->nb;
  p->rec_cap = 4096;
  auto cleanup = [&](mf_status s) {
    mf_process_destroy(p);
    return s;
  };
  if (hipMalloc(&p->d_pdf, sizeof(double) * 16 * NXK) != hipSuccess ||
      hipMalloc(&p->d_edges, sizeof(double) * p->ndim * (p->nb + 1)) != hipSuccess ||
      hipMalloc(&p->d_part, sizeof(double) * (size_t)MAX_BLOCKS * std::max(p->pstride, 3 * GV)) != hipSuccess ||
      hipMalloc(&p->d_part2, sizeof(double) * (size_t)RED_ROWS * p->pstride) != hipSuccess ||
      hipMalloc(&p->d_rec, sizeof(double) * REC * p->rec_cap) != hipSuccess ||
      hipMalloc(&p->d_hist, sizeof(double) * p->ndim * p->nb) != hipSuccess ||
      hipMalloc(&p->d_out, sizeof(double) * 64) != hipSuccess ||
      hipMalloc(&p->d_status, sizeof(int) * 4) != hipSuccess) {
    hipGetLastError();
    return cleanup(fail(MF_ENOMEM, "device allocation failed"));
  }
  c.pdfc = p->d_pdf;
  c.pdfd = p->d_pdf + 4 * NXK;
  c.pdft = p->d_pdf + 8 * NXK;
  PdfParams P;
  for (int i = 0; i < 20; ++i) P.p[i] = cfg->pdf_params[i];
  hipLaunchKernelGGL(k_pdf_setup, dim3((4 * NXK + 255) / 256), dim3(256), 0, 0, P, mu, p->d_pdf, p->d_pdf + 4 * NXK,
                     p->d_pdf + 8 * NXK);
  hipLaunchKernelGGL(k_fill_uniform, dim3((p->ndim * (p->nb + 1) + 255) / 256), dim3(256), 0, 0, p->d_edges,
                     p->ndim, p->nb);
  if (c.dyn_scale) {
    if (hipMalloc(&p->d_pdfq, sizeof(double) * 4 * NQK * NXK) != hipSuccess) {
      hipGetLastError();
      return cleanup(fail(MF_ENOMEM, "device allocation failed"));
    }
    c.pdfq = p->d_pdfq;
    hipLaunchKernelGGL(k_pdf_table, dim3((4 * NQK * NXK + 255) / 256), dim3(256), 0, 0, P, p->d_pdfq);
  }
  if (hipDeviceSynchronize() != hipSuccess) return cleanup(fail(MF_EDEVICE, "table set-up failed"));
  *out = p;
  return MF_OK;
}

void mf_process_destroy(mf_process* p) {
  if (!p) return;
  hipFree(p->d_pdf);
  hipFree(p->d_edges);
  hipFree(p->d_part);
  hipFree(p->d_part2);
  hipFree(p->d_rec);
  hipFree(p->d_hist);
  hipFree(p->d_out);
  hipFree(p->d_status);
  hipFree(p->d_sx);
  hipFree(p->d_sjac);
  hipFree(p->d_sw);
  hipFree(p->d_sbins);
  hipFree(p->d_sy);
  hipFree(p->d_slq);
  hipFree(p->d_sz);
  hipFree(p->d_sw32);
  if (p->ws && p->L.ws_free) p->L.ws_free(p->ws);
  hipFree(p->d_sel);
  hipFree(p->d_selcnt);
  hipFree(p->d_selw);
  hipFree(p->d_obs);
  hipFree(p->d_pdfq);
  delete p;
}

mf_status mf_integrand(mf_process* p, const double* u, int64_t n, double* w, void* stream) {
  mf::clear_error();
  if (!p) return fail(MF_EINVAL, "NULL process");
  if (n < 0) return fail(MF_EINVAL, "negative event count");
  if (n == 0) return MF_OK;
  if (!u || !w) return fail(MF_EINVAL, "NULL buffer");
  return run_integrand(p, u, n, w, (hipStream_t)stream);
}

mf_status mf_integrand_noalloc(mf_process* p, const double* u, int64_t n, double* w, void* stream) {
  mf::clear_error();
  if (!p) return fail(MF_EINVAL, "NULL process");
  if (n < 0) return fail(MF_EINVAL, "negative event count");
  if (n == 0) return MF_OK;
  if (!u || !w) return fail(MF_EINVAL, "NULL buffer");
  if (n > NOALLOC_MAX_POINTS)
    return fail(MF_EINVAL, "mf_integrand_noalloc takes at most %lld points per call (got %lld)",
                (long long)NOALLOC_MAX_POINTS, (long long)n);
  if (p->L.integrand_ws || !p->L.integrand)
    return fail(MF_ENOTSUP, "this process evaluates its integrand with a multi-kernel workspace; use mf_integrand");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != p->device) return fail(MF_EINVAL, "the process was created on device %d, current is %d", p->device, dev);
  if (dev < 0 || dev >= MAX_DEVICES || !g_noalloc_ptr[dev])
    return fail(MF_EDEVICE, "scratch array address unavailable on device %d: %s", dev,
                hipGetErrorString(dev >= 0 && dev < MAX_DEVICES ? g_noalloc_err[dev] : hipErrorInvalidDevice));
  const int nblk = blocks_for(n);
  const int64_t cap = (n + (int64_t)nblk * BLOCK - 1) / ((int64_t)nblk * BLOCK) * BLOCK;
  int* cnt = g_noalloc_ptr[dev];
  int* list = cnt + MAX_BLOCKS;  // nblk * cap <= NOALLOC_MAX_POINTS entries (see the array's bound)
  p->L.integrand(p->dc, u, n, w, nblk, list, cnt, cap, (hipStream_t)stream);
  return check_stream_launch("k_integrand");
}

mf_status mf_integrand_grad(mf_process* p, const double* u, int64_t n, double* w, double* dw, void* stream) {
  mf::clear_error();
  if (!p) return fail(MF_EINVAL, "NULL process");
  if (n < 0) return fail(MF_EINVAL, "negative event count");
  if (n == 0) return MF_OK;
  if (!u || !dw) return fail(MF_EINVAL, "NULL buffer");
  hipStream_t s = (hipStream_t)stream;
  const int nblk = blocks_for(n);
  if (!p->L.integrand_grad) return fail(MF_ENOTSUP, "derivatives are not built for this process");
  if (p->dc.dyn_scale) return fail(MF_ENOTSUP, "derivatives are not built with the dynamic scale");
  p->L.integrand_grad(p->dc, u, n, w, dw, nblk, s);
  return check_stream_launch("k_integrand_grad");
}

mf_status mf_vegas_refine(double* edges, const double* hist, int ndim, int nbins, double alpha, int32_t* status,
                          void* stream) {
  mf::clear_error();
  if (!edges || !hist || !status) return fail(MF_EINVAL, "NULL buffer");
  if (ndim < 1 || ndim > MAXD) return fail(MF_EINVAL, "ndim must be in 1..%d", MAXD);
  if (nbins < 1 || nbins > MAX_BINS) return fail(MF_EINVAL, "nbins must be in 1..%d", MAX_BINS);
  if (!(alpha > 0.0)) return fail(MF_EINVAL, "alpha must be positive");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_clear_status, dim3(1), dim3(1), 0, s, status);
  hipLaunchKernelGGL(k_refine, dim3(ndim), dim3(64), 0, s, edges, hist, ndim, nbins, alpha, status);
  int hs = 0;
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(&hs, status, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (hs) return fail(MF_ERANGE, "refined grid not strictly increasing; dimension left unchanged");
  return MF_OK;
}

mf_status mf_integrate(mf_process* p, const mf_integrate_opts* o, mf_result* r) {
  mf::clear_error();
  if (!p || !o || !r) return fail(MF_EINVAL, "NULL argument");
  if (o->n_iter < 1 || o->n_iter > p->rec_cap) return fail(MF_EINVAL, "n_iter must be in 1..%d", p->rec_cap);
  if (o->n_events < 2) return fail(MF_EINVAL, "n_events must be >= 2");
  if (o->warmup_iters_discarded < 0 || o->warmup_iters_discarded >= o->n_iter)
    return fail(MF_EINVAL, "warmup_iters_discarded must be in 0..n_iter-1");
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = (hipStream_t)o->stream;
  const int d = p->ndim, nb = p->nb;
  if (o->edges_in) HIP_TRY(hipMemcpyAsync(p->d_edges, o->edges_in, sizeof(double) * d * (nb + 1),
                                          hipMemcpyDeviceToDevice, s));
  const int nblk = iter_blocks(o->n_events);
  const size_t lds = vegas_lds_bytes(d, nb);
  if (o->flow) {
    if (o->adapt) return fail(MF_EINVAL, "the grid is frozen under a flow proposal (adapt must be 0)");
    if (!(o->flow_mix >= 0.0 && o->flow_mix < 1.0)) return fail(MF_EINVAL, "flow_mix must be in [0,1)");
    if (mf_flow_ndim(o->flow) != d) return fail(MF_EINVAL, "flow dimension differs from the integrand's");
  }
  if (!(o->fallback_rel_var >= 0.0) || !std::isfinite(o->fallback_rel_var))
    return fail(MF_EINVAL, "fallback_rel_var must be finite and >= 0");
  const bool can_fallback = o->flow && o->fallback_rel_var > 0.0;
  if (!p->L.fused || o->flow) {
    mf_status st = ensure_stage(p, o->n_events, s);
    if (st != MF_OK) return st;
  }
  if (p->L.fused && (!o->flow || can_fallback)) {
    mf_status st = ensure_select(p, o->n_events, nblk, s);
    if (st != MF_OK) return st;
  }
  // the proposal of the current iteration: the flow until a fallback
  mf_flow* flow = o->flow;
  int fallback_iter = -1;
  double flow_rv = -1.0;
  // observable histograms: validation and buffers
  ObsSpec ospec{};
  const int OW = o->obs ? N_OBS * o->obs->nbins * 2 : 0;  // histogram row width
  if (o->obs) {
    const mf_observables* ob = o->obs;
    if (o->flow || !p->L.fused || !p->L.observables)
      return fail(MF_ENOTSUP, "observable histograms are built for VEGAS iterations of the single-kernel processes");
    if (ob->nbins < 1 || ob->nbins > MAX_OBS_BINS) return fail(MF_EINVAL, "nbins must be in 1..%d", MAX_OBS_BINS);
    if (!ob->sums) return fail(MF_EINVAL, "NULL histogram output");
    ospec.nbins = ob->nbins;
    for (int q = 0; q < N_OBS; ++q) {
      if (!(std::isfinite(ob->lo[q]) && std::isfinite(ob->hi[q]) && ob->hi[q] > ob->lo[q]))
        return fail(MF_EINVAL, "observable %d: need finite lo < hi", q);
      ospec.lo[q] = ob->lo[q];
      ospec.scale[q] = ob->nbins / (ob->hi[q] - ob->lo[q]);
    }
    if (p->selw_cap < p->sel_cap) {
      HIP_TRY(hipStreamSynchronize(s));
      (void)hipFree(p->d_selw);
      p->d_selw = nullptr;
      p->selw_cap = 0;
      if (hipMalloc(&p->d_selw, sizeof(double) * (size_t)MAX_BLOCKS * p->sel_cap) != hipSuccess)
        return fail(MF_ENOMEM, "weights of the kept events");
      p->selw_cap = p->sel_cap;
    }
    if (!p->d_obs && hipMalloc(&p->d_obs, sizeof(double) * (size_t)(MAX_BLOCKS + RED_ROWS + 1) * N_OBS *
                                              MAX_OBS_BINS * 2) != hipSuccess)
      return fail(MF_ENOMEM, "observable partials");
    HIP_TRY(hipMemsetAsync(p->d_obs + (size_t)(MAX_BLOCKS + RED_ROWS) * OW, 0, sizeof(double) * OW, s));
  }
  std::vector<double> rec((size_t)REC * o->n_iter, 0.0);
  double time_to_target = -1.0;
  int done = 0;
  std::vector<hipEvent_t> ev(2 * (size_t)o->n_iter);
  for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
  struct EvGuard {
    std::vector<hipEvent_t>& v;
    ~EvGuard() {
      for (auto& e : v) (void)hipEventDestroy(e);
    }
  } guard{ev};
  double sw = 0.0, swi = 0.0;
  if (o->prior && o->prior->error > 0.0) {
    sw = 1.0 / (o->prior->error * o->prior->error);
    swi = o->prior->integral * sw;
  }
  for (int it = 0; it < o->n_iter; ++it) {
    const uint64_t iter = o->iter_offset + (uint64_t)it;
    HIP_TRY(hipEventRecord(ev[2 * it], s));
    if (flow) {
      const int64_t N = o->n_events;
      mf_status sst = stage_sample(p, flow, o->flow_mix, iter, N, nullptr, s);
      if (sst != MF_OK) return sst;
      sst = run_integrand(p, p->d_sx, N, p->d_sw, s);
      if (sst != MF_OK) return sst;
      hipLaunchKernelGGL(k_stage_accumulate, dim3(nblk), dim3(256), 0, s, p->d_sw, p->d_sjac, p->d_sbins, d, nb, N,
                         p->d_part, p->pstride);
    } else if (p->L.fused) {
      p->L.vegas(p->dc, p->d_edges, iter, o->n_events, p->cfg.seed, p->d_part, p->pstride, nblk, lds, p->d_sel,
                 p->d_selcnt, p->sel_cap, o->obs ? p->d_selw : nullptr, s);
      if (o->obs && it >= o->warmup_iters_discarded) {
        double* opart = p->d_obs;
        double* orows = p->d_obs + (size_t)MAX_BLOCKS * OW;
        double* osums = p->d_obs + (size_t)(MAX_BLOCKS + RED_ROWS) * OW;
        p->L.observables(p->dc, p->d_edges, iter, p->cfg.seed, p->d_sel, p->d_selcnt, p->sel_cap, p->d_selw, ospec,
                         opart, nblk, s);
        const int R = nblk < RED_ROWS ? nblk : RED_ROWS;
        hipLaunchKernelGGL(k_obs_reduce, dim3((OW + 255) / 256, R), dim3(256), 0, s, opart, nblk, OW, R, orows);
        hipLaunchKernelGGL(k_obs_accumulate, dim3((OW + 255) / 256), dim3(256), 0, s, orows, R, OW, osums);
      }
    } else {
      const int64_t N = o->n_events;
      hipLaunchKernelGGL(k_stage_points, dim3(nblk), dim3(256), sizeof(double) * d * (nb + 1), s, p->d_edges, d, nb,
                         iter, N, p->cfg.seed, p->d_sx, p->d_sjac, p->d_sbins);
      mf_status sst = run_integrand(p, p->d_sx, N, p->d_sw, s);
      if (sst != MF_OK) return sst;
      hipLaunchKernelGGL(k_stage_accumulate, dim3(nblk), dim3(256), 0, s, p->d_sw, p->d_sjac, p->d_sbins, d, nb, N,
                         p->d_part, p->pstride);
    }
    HIP_TRY(hipEventRecord(ev[2 * it + 1], s));
    mf_status st = check_stream_launch("k_vegas");
    if (st != MF_OK) return st;
    const int R = nblk < RED_ROWS ? nblk : RED_ROWS;
    hipLaunchKernelGGL(k_reduce_partials, dim3(R), dim3(256), 0, s, p->d_part, nblk, p->pstride, PART_HEAD + d * nb,
                       R, p->d_part2);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, s, p->d_part2, R, p->pstride, d, nb, o->n_events,
                       p->cfg.alpha, o->adapt ? 1 : 0, p->d_edges, p->d_rec + (size_t)REC * it, p->d_hist);
    st = check_stream_launch("k_finalize");
    if (st != MF_OK) return st;
    done = it + 1;
    const bool test_fallback = can_fallback && it == 0;
    if (o->target_rel_err > 0.0 || test_fallback) {
      HIP_TRY(hipMemcpyAsync(rec.data() + (size_t)REC * it, p->d_rec + (size_t)REC * it, sizeof(double) * REC,
                             hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
    }
    if (r->iter_seconds)
      r->iter_seconds[it] = o->target_rel_err > 0.0
                                ? std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count()
                                : 0.0;
    if (test_fallback) {
      // per-event relative variance of the flow's first iteration against
      // the VEGAS proposal's on the same frozen grid
      const double* q = rec.data() + (size_t)REC * it;
      const double n1 = (double)(o->n_events - 1);
      flow_rv = q[0] != 0.0 ? n1 * q[1] * q[1] / (q[0] * q[0]) : INFINITY;
      if (!(flow_rv <= o->fallback_rel_var)) {
        flow = nullptr;
        fallback_iter = it + 1;
      }
    }
    if (o->target_rel_err > 0.0) {
      const double* q = rec.data() + (size_t)REC * it;
      if (it >= o->warmup_iters_discarded && q[1] > 0.0) {
        sw += 1.0 / (q[1] * q[1]);
        swi += q[0] / (q[1] * q[1]);
      }
      if (sw > 0.0) {
        double mean = swi / sw, err = std::sqrt(1.0 / sw);
        if (mean != 0.0 && err / std::fabs(mean) <= o->target_rel_err) {
          time_to_target = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
          break;
        }
      }
    }
  }
  HIP_TRY(hipMemcpyAsync(rec.data(), p->d_rec, sizeof(double) * REC * done, hipMemcpyDeviceToHost, s));
  if (o->edges_out)
    HIP_TRY(hipMemcpyAsync(o->edges_out, p->d_edges, sizeof(double) * d * (nb + 1), hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  // combination of the iteration estimates (inverse-variance weights)
  double W = 0.0, WI = 0.0, nz = 0.0, bad = 0.0;
  int k = 0;
  const bool has_prior = o->prior && o->prior->error > 0.0;
  if (has_prior) {
    W = 1.0 / (o->prior->error * o->prior->error);
    WI = o->prior->integral * W;
    ++k;
  }
  for (int it = 0; it < done; ++it) {
    const double* q = rec.data() + (size_t)REC * it;
    nz += q[4];
    bad += q[5];
    if (r->iter_integral) r->iter_integral[it] = q[0];
    if (r->iter_error) r->iter_error[it] = q[1];
    if (it < o->warmup_iters_discarded || !(q[1] > 0.0)) continue;
    W += 1.0 / (q[1] * q[1]);
    WI += q[0] / (q[1] * q[1]);
    ++k;
  }
  double mean = W > 0.0 ? WI / W : 0.0;
  double chi2 = 0.0;
  if (has_prior) chi2 += (o->prior->integral - mean) * (o->prior->integral - mean) / (o->prior->error * o->prior->error);
  for (int it = o->warmup_iters_discarded; it < done; ++it) {
    const double* q = rec.data() + (size_t)REC * it;
    if (q[1] > 0.0) chi2 += (q[0] - mean) * (q[0] - mean) / (q[1] * q[1]);
  }
  r->integral = mean;
  r->error = W > 0.0 ? std::sqrt(1.0 / W) : 0.0;
  r->chi2_dof = k > 1 ? chi2 / (k - 1) : 0.0;
  r->n_iter_done = done;
  r->n_events_total = (int64_t)done * o->n_events;
  r->n_nonzero = (int64_t)nz;
  r->n_nonfinite = (int64_t)bad;
  r->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  r->time_to_target = time_to_target;
  double ksec = 0.0;
  for (int it = 0; it < done; ++it) {
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, ev[2 * it], ev[2 * it + 1]));
    ksec += 1e-3 * ms;
  }
  r->kernel_seconds = ksec;
  r->fallback_iter = fallback_iter < done ? fallback_iter : -1;
  r->flow_rel_var = flow_rv;
  for (int it = 0; it < done; ++it)
    if (rec[(size_t)REC * it + 6] != 0.0) return fail(MF_ERANGE, "grid refinement failed at iteration %d", it);
  if (o->obs) {
    HIP_TRY(hipMemcpyAsync(o->obs->sums, p->d_obs + (size_t)(MAX_BLOCKS + RED_ROWS) * OW, sizeof(double) * OW,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (o->obs->sigma) {
      // per-bin cross section and Monte Carlo error over the counted events
      const double M = (double)o->n_events * (double)std::max(done - o->warmup_iters_discarded, 0);
      for (int b = 0; b < OW / 2; ++b) {
        const double mean = M > 0.0 ? o->obs->sums[2 * b] / M : 0.0;
        const double var = M > 1.0 ? (o->obs->sums[2 * b + 1] / M - mean * mean) / (M - 1.0) : 0.0;
        o->obs->sigma[2 * b] = mean;
        o->obs->sigma[2 * b + 1] = std::sqrt(std::max(var, 0.0));
      }
    }
  }
  // the integrand never returns a non-finite value, so under a learned
  // proposal a non-finite weight comes from the proposal's density: the
  // estimate would silently miss those points
  if (o->flow && bad > 0.0)
    return fail(MF_ERANGE, "the proposal gave %.0f non-finite weights (diverged training)", bad);
  return MF_OK;
}

mf_status mf_weights(mf_process* p, mf_flow* flow, double flow_mix, uint64_t iter, int64_t n, float* y_out,
                     double* w_out, void* stream) {
  mf::clear_error();
  if (!p) return fail(MF_EINVAL, "NULL process");
  if (flow && !(flow_mix >= 0.0 && flow_mix < 1.0)) return fail(MF_EINVAL, "flow_mix must be in [0,1)");
  if (n < 0) return fail(MF_EINVAL, "negative event count");
  if (n == 0) return MF_OK;
  if (!w_out) return fail(MF_EINVAL, "NULL weight buffer");
  if (flow && mf_flow_ndim(flow) != p->ndim) return fail(MF_EINVAL, "flow dimension differs from the integrand's");
  hipStream_t s = (hipStream_t)stream;
  mf_status st = ensure_stage(p, n, s);
  if (st != MF_OK) return st;
  st = stage_sample(p, flow, flow_mix, iter, n, y_out, s);
  if (st != MF_OK) return st;
  st = run_integrand(p, p->d_sx, n, p->d_sw, s);
  if (st != MF_OK) return st;
  hipLaunchKernelGGL(k_weight, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p->d_sw, p->d_sjac, n, w_out);
  return check_stream_launch("k_weight");
}

namespace {
// Inverse-variance combination of iteration estimates (integral, error),
// optionally starting from a prior estimate; chi^2 per degree of freedom.
struct Combo {
  double W = 0.0, WI = 0.0;
  std::vector<double> I, E;
  void add(double i, double e) {
    I.push_back(i);
    E.push_back(e);
    if (e > 0.0) {
      W += 1.0 / (e * e);
      WI += i / (e * e);
    }
  }
  double mean() const { return W > 0.0 ? WI / W : 0.0; }
  double error() const { return W > 0.0 ? std::sqrt(1.0 / W) : 0.0; }
  double chi2_dof() const {
    double m = mean(), c = 0.0;
    int k = 0;
    for (size_t j = 0; j < I.size(); ++j)
      if (E[j] > 0.0) {
        c += (I[j] - m) * (I[j] - m) / (E[j] * E[j]);
        ++k;
      }
    return k > 1 ? c / (k - 1) : 0.0;
  }
};
}  // namespace

mf_status mf_flow_train_online(mf_process* p, mf_flow* flow, const mf_flow_online_opts* o, double* loss_per_step,
                               mf_result* est) {
  mf::clear_error();
  auto t0 = std::chrono::steady_clock::now();
  if (!p || !flow || !o) return fail(MF_EINVAL, "NULL argument");
  if (mf_flow_ndim(flow) != p->ndim) return fail(MF_EINVAL, "flow dimension differs from the integrand's");
  if (o->steps < 1) return fail(MF_EINVAL, "steps must be >= 1");
  if (o->batch < 2) return fail(MF_EINVAL, "batch must be >= 2");
  if (!(o->flow_mix >= 0.0 && o->flow_mix < 1.0)) return fail(MF_EINVAL, "flow_mix must be in [0,1)");
  if (!(o->lr > 0.0) || !(o->lr_final >= 0.0)) return fail(MF_EINVAL, "invalid learning rates");
  if (o->loss != MF_FLOW_LOSS_KL && o->loss != MF_FLOW_LOSS_VARIANCE) return fail(MF_EINVAL, "unknown loss %d", o->loss);
  if (o->group_steps < 0 || !(o->target_rel_err >= 0.0)) return fail(MF_EINVAL, "invalid grouping or target");
  hipStream_t s = (hipStream_t)o->stream;
  const int64_t n = o->batch;
  const int group = o->group_steps > 0 ? o->group_steps : o->steps;
  mf_status st = ensure_stage(p, n, s);
  if (st != MF_OK) return st;
  float* d_loss = nullptr;
  double* d_sums = nullptr;  // [steps][2] batch sums, then one int flag
  HIP_TRY(hipMalloc(&d_loss, sizeof(float) * 2 * o->steps));
  if (hipMalloc(&d_sums, sizeof(double) * (2 * o->steps + 1)) != hipSuccess) {
    (void)hipFree(d_loss);
    return fail(MF_ENOMEM, "training statistics");
  }
  struct Free {
    float* q;
    double* r;
    ~Free() {
      (void)hipFree(q);
      (void)hipFree(r);
    }
  } guard{d_loss, d_sums};
  int* d_bad = reinterpret_cast<int*>(d_sums + 2 * o->steps);
  HIP_TRY(hipMemsetAsync(d_bad, 0, sizeof(int), s));
  float* wt = p->d_sw32;
  float* rw = p->d_sw32 + n;
  float* r2 = p->d_sw32 + 2 * n;
  Combo combo;
  std::vector<double> hs(2 * (size_t)o->steps);
  double time_to_target = -1.0;
  int done = 0, g0 = 0;
  for (int t = 0; t < o->steps; ++t) {
    st = stage_sample(p, flow, o->flow_mix, o->iter_offset + (uint64_t)t, n, nullptr, s);
    if (st != MF_OK) return st;
    st = run_integrand(p, p->d_sx, n, p->d_sw, s);
    if (st != MF_OK) return st;
    hipLaunchKernelGGL(k_online_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p->d_sw, p->d_sjac,
                       p->d_slq, o->flow_mix, n, o->loss == MF_FLOW_LOSS_VARIANCE ? 1 : 0, wt, rw, r2, d_bad);
    hipLaunchKernelGGL(k_batch_relvar, dim3(1), dim3(1024), 0, s, rw, r2, n, d_loss + 2 * t, d_sums + 2 * t);
    const double lr =
        o->lr_final + 0.5 * (o->lr - o->lr_final) * (1.0 + std::cos(M_PI * (double)t / (double)o->steps));
    st = mf::flow_step(flow, p->d_sy, n, wt, n, d_loss + 2 * t + 1, lr, s);
    if (st != MF_OK) return st;
    done = t + 1;
    if (done - g0 == group || done == o->steps) {
      // the group's estimate: all its batches pooled (each batch is an unbiased
      // sample of the integral from the flow as it was at that step)
      int h_bad = 0;
      HIP_TRY(hipMemcpyAsync(hs.data() + 2 * (size_t)g0, d_sums + 2 * g0, sizeof(double) * 2 * (done - g0),
                             hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(&h_bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      if (h_bad)
        return fail(MF_ERANGE, "the proposal gave non-finite densities by step %d (diverged training; "
                               "lower the learning rate)", done);
      double S1 = 0.0, S2 = 0.0;
      for (int k = g0; k < done; ++k) {
        S1 += hs[2 * (size_t)k];
        S2 += hs[2 * (size_t)k + 1];
      }
      const double N = (double)(done - g0) * (double)n;
      const double I = S1 / N, var = (S2 / N - I * I) / (N - 1.0);
      combo.add(I, std::sqrt(var > 0.0 ? var : 0.0));
      g0 = done;
      if (o->target_rel_err > 0.0 && combo.mean() != 0.0 &&
          combo.error() / std::fabs(combo.mean()) <= o->target_rel_err) {
        time_to_target = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        break;
      }
    }
  }
  std::vector<float> hl(2 * (size_t)o->steps);
  HIP_TRY(hipMemcpyAsync(hl.data(), d_loss, sizeof(float) * 2 * done, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (loss_per_step)
    for (int t = 0; t < o->steps; ++t) loss_per_step[t] = t < done ? hl[2 * (size_t)t] : 0.0;
  if (est) {
    est->integral = combo.mean();
    est->error = combo.error();
    est->chi2_dof = combo.chi2_dof();
    est->n_iter_done = (int32_t)combo.I.size();
    est->n_events_total = (int64_t)done * n;
    est->n_nonzero = 0;
    est->n_nonfinite = 0;
    est->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    est->time_to_target = time_to_target;
    est->kernel_seconds = 0.0;
    est->fallback_iter = -1;
    est->flow_rel_var = -1.0;
    for (size_t j = 0; j < combo.I.size(); ++j) {
      if (est->iter_integral) est->iter_integral[j] = combo.I[j];
      if (est->iter_error) est->iter_error[j] = combo.E[j];
    }
  }
  return MF_OK;
}

mf_status mf_grad(mf_process* p, const mf_integrate_opts* o, double* out, double* err) {
  mf::clear_error();
  if (!p || !o || !out || !err) return fail(MF_EINVAL, "NULL argument");
  if (o->n_events < 2) return fail(MF_EINVAL, "n_events must be >= 2");
  hipStream_t s = (hipStream_t)o->stream;
  const int d = p->ndim, nb = p->nb;
  if (o->edges_in) HIP_TRY(hipMemcpyAsync(p->d_edges, o->edges_in, sizeof(double) * d * (nb + 1),
                                          hipMemcpyDeviceToDevice, s));
  const int nblk = blocks_for(o->n_events);
  const size_t lds = sizeof(double) * (d * (nb + 1) + WAVES * GV * 4);
  if (!p->L.grad_vegas) return fail(MF_ENOTSUP, "derivatives are not built for this process");
  if (p->dc.dyn_scale) return fail(MF_ENOTSUP, "derivatives are not built with the dynamic scale");
  mf_status sst = ensure_select(p, o->n_events, nblk, s);
  if (sst != MF_OK) return sst;
  p->L.grad_vegas(p->dc, p->d_edges, o->iter_offset, o->n_events, p->cfg.seed, p->d_part, nblk, lds, p->d_sel,
                  p->d_selcnt, p->sel_cap, s);
  mf_status st = check_stream_launch("k_grad_vegas");
  if (st != MF_OK) return st;
  hipLaunchKernelGGL(k_grad_finalize, dim3(1), dim3(64), 0, s, p->d_part, nblk, o->n_events, p->d_out);
  double h[2 * GV];
  HIP_TRY(hipMemcpyAsync(h, p->d_out, sizeof(h), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int k = 0; k < GV; ++k) {
    out[k] = h[k];
    err[k] = h[GV + k];
  }
  return MF_OK;
}

}  // extern "C"
