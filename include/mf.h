/*
 * mf.h -- C ABI of the MI355X (gfx950) per-event LO integrand library.
 *
 * The library evaluates, entirely in HIP kernels, the event pipeline of a
 * parton-level Monte Carlo described in arXiv:2105.10529, Sec. 2.1 (random
 * numbers -> phase-space kinematics with fiducial cuts -> PDFs -> matrix
 * element -> histogram accumulation for the VEGAS grid), with the helicity
 * loop and the aggregation of colour-ordered amplitudes of Sec. 2.2.
 * Processes: g g -> t t~ + 0..3 gluons and q q~ -> t t~ (q = u, d).
 *
 * Conventions shared by every call:
 *  - Every call returns mf_status; MF_OK is 0.  On error a description is
 *    available from mf_last_error() (thread-local, valid until the next call
 *    on the same thread).  No C++ exception crosses this interface.
 *  - Pointers documented as "device" are HIP device pointers (for example
 *    torch.Tensor.data_ptr() of a cuda tensor); "host" pointers are ordinary
 *    host memory.  The caller owns every buffer it passes.  The library
 *    allocates device memory only inside an mf_process handle (tables, the
 *    VEGAS grid, reduction partials, staging buffers) and frees it in
 *    mf_process_destroy; the calls without a handle (mf_vegas_refine,
 *    mf_weight_stats, mf_vjp) work in scratch the caller passes.
 *  - g g -> t t~ g g g (and g g -> t t~ g g with the matrix-core colour
 *    form) evaluates the integrand in stages: kinematics and cuts, then the
 *    partial amplitudes of the events that pass, streamed through a
 *    handle-owned buffer of up to 2 GiB, then the colour sum on the matrix
 *    cores.  These integrand calls synchronise `stream` once (to read the
 *    number of passing events).
 *  - `stream` is a hipStream_t passed as void*; NULL means the default
 *    stream.  Calls taking a stream are asynchronous with respect to the
 *    host unless stated otherwise.
 *  - For fixed inputs (seed, event count, configuration) results are
 *    bitwise reproducible: reductions run in a fixed order.
 *  - Units: GeV for energies and masses, pb for cross sections.
 */
#ifndef MF_H
#define MF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MF_OK = 0,
  MF_EINVAL = 1,   /* invalid argument or non-physical configuration */
  MF_ERANGE = 2,   /* value outside a supported range (grid order, PDF range) */
  MF_ENOMEM = 3,   /* device allocation failed */
  MF_EDEVICE = 4,  /* HIP runtime error (launch, copy, synchronisation) */
  MF_ENOTSUP = 5   /* combination not provided by the library */
} mf_status;

typedef enum {
  MF_GG_TTX = 0,     /* g g -> t t~                         (4 dims)  */
  MF_UUX_TTX = 1,    /* u u~ -> t t~, both beam assignments  (4 dims)  */
  MF_DDX_TTX = 2,    /* d d~ -> t t~, both beam assignments  (4 dims)  */
  MF_GG_TTXG = 3,    /* g g -> t t~ g                        (7 dims)  */
  MF_GG_TTXGG = 4,   /* g g -> t t~ g g                      (10 dims) */
  MF_GG_TTXGGG = 5,  /* g g -> t t~ g g g                    (13 dims) */
  MF_UUX_TTXG = 6,   /* u u~ -> t t~ g, both beam assignments (7 dims) */
  MF_DDX_TTXG = 7,   /* d d~ -> t t~ g, both beam assignments (7 dims) */
  MF_QG_TTXQ = 8     /* q g -> t t~ q and q~ g -> t t~ q~ for q = u, d,
                        both beam assignments (7 dims); the cuts act on
                        the final light quark as on a gluon */
} mf_process_id;

typedef enum {
  MF_PREC_FP64 = 0,     /* every step in FP64 */
  MF_PREC_FP32_AMP = 1  /* amplitudes in FP32; kinematics, PDFs, weights
                           and all accumulations in FP64 */
} mf_precision;

/* Configuration of one integrand (create-time; immutable afterwards). */
typedef struct {
  int32_t process;         /* mf_process_id */
  int32_t precision;       /* mf_precision */
  double sqrt_s;           /* hadronic centre-of-mass energy, > 2 m_t */
  double m_t;              /* top mass, > 0 */
  double mu;               /* factorisation scale; <= 0 selects mu = m_t */
  double alpha_s;          /* fixed strong coupling, > 0 */
  double pt_min;           /* gluon cut pT > pt_min (GeV) */
  double eta_max;          /* gluon cut |eta| < eta_max (lab frame) */
  double dr_min;           /* gluon-gluon cut dR > dr_min; <= 0 disables */
  double pdf_params[20];   /* (A, a, b, c, d) of x f = A x^(a+bL) (1-x)^(c+dL),
                              L = ln(Q/1.65 GeV), for g, u, d, u~ (d~ = u~) */
  int32_t n_bins;          /* VEGAS bins per dimension, 1..64 */
  double alpha;            /* VEGAS refinement damping exponent, > 0 */
  uint64_t seed;           /* Philox key word 0 for in-library sampling */
  int32_t helicity;        /* polarisation states of g g -> t t~ g g g (other
                              processes: 0 only, else MF_ENOTSUP):
                              0 = sum over all 64 states (antitop helicity x
                                  gluon polarisations; both top helicities
                                  always summed);
                              1 = one state per point, drawn by Philox4x64-10
                                  from the point itself (counter = the bit
                                  patterns of its first two coordinates, key
                                  (seed, 5)), weighted by 64: an unbiased
                                  estimate of the sum at 1/64 of the amplitude
                                  work;
                              2 + k = only state k (0..63), weight not scaled
                                  (the 64 single-state integrands add up to
                                  the sum; for checks) */
  int32_t dynamic_scale;   /* 0: the fixed scale mu above; 1: per event
                              mu = H_T / 2, half the sum of the final-state
                              transverse masses (tops of mass m_t, massless
                              gluons), with the PDFs interpolated in x and Q
                              on the full knot grid (the derivative entry
                              points are then MF_ENOTSUP) */
  int32_t colour_form;     /* colour quadratic form of g g -> t t~ g g (other
                              processes: 0 only, else MF_ENOTSUP):
                              0 = the default, 1 (the faster form in both
                                  precisions);
                              1 = in registers on the vector ALUs, next to
                                  the amplitudes (FP32: one fused kernel per
                                  VEGAS iteration; FP64: points, integrand
                                  and accumulation kernels);
                              2 = on the matrix cores: the partial amplitudes
                                  are streamed to a handle-owned buffer and
                                  Z = C A is formed with FP32 (FP64)
                                  matrix-core products, then A . Z */
} mf_config;

typedef struct mf_process mf_process;

/* Create an integrand on the current HIP device: validates cfg, tabulates
 * the PDF grid (196 points uniform in ln x over [1e-9, 1] x 50 points
 * uniform in ln Q over [1.65, 1e5] GeV) and collapses it at the fixed scale,
 * allocates the VEGAS grid (uniform).  *out receives the handle.
 * MF_EINVAL for sqrt_s <= 2 m_t, non-positive masses/couplings, a scale
 * outside the Q grid or an unknown process; MF_ENOTSUP for a precision the
 * process does not provide (the quark channels: FP64 only);
 * MF_ENOMEM / MF_EDEVICE on HIP failures. */
mf_status mf_process_create(const mf_config* cfg, mf_process** out);

/* Release every device allocation of the handle (NULL is accepted). */
void mf_process_destroy(mf_process* p);

/* Number of integration dimensions: 4, 7, 10 or 13 (3 n_final - 2). */
int mf_process_ndim(const mf_process* p);

/* Thread-local description of the last error ("" if none). */
const char* mf_last_error(void);

/* The integrand at caller-supplied points (the phase-space, PDF and matrix
 * element part of the event pipeline, Sec. 2.1, without the VEGAS map):
 *   u: device, [ndim][n] FP64 structure of arrays, each value in (0,1):
 *      u[0], u[1] are the momentum fractions x1, x2; then the n_final-2
 *      intermediate-mass uniforms; then (cos theta, phi) uniforms per two-body
 *      split, the t t~ split last.
 *   w: device, [n] FP64 output: d sigma in pb per unit hypercube volume.
 *      Zero below threshold or outside the cuts; a non-finite value is
 *      never written (such events give 0).
 * Points that fail threshold or cuts are written as 0 without evaluating the
 * matrix element.  The call may allocate (or grow) per-block point lists
 * inside the handle (4 B per point), synchronising `stream` when it does.
 * n = 0 is accepted and does nothing.  MF_EINVAL for n < 0, n >= 2^31 or NULL
 * pointers with n > 0. */
mf_status mf_integrand(mf_process* p, const double* u, int64_t n, double* w, void* stream);

/* mf_integrand for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same results, bit for bit, as mf_integrand, with
 * the per-block point lists in a fixed device array of the library
 * (16 MiB per device, held until the process ends) instead of the handle.
 * No device memory is allocated or freed.  At most MF_NOALLOC_MAX_POINTS
 * points per call (MF_EINVAL above); MF_ENOTSUP where the integrand runs as
 * several kernels with a workspace (g g -> t t~ g g g, and g g -> t t~ g g
 * with the matrix-core colour form); MF_EINVAL if the current device is not
 * the handle's.
 * Every call on a device shares that device's array, so calls that overlap
 * on one device (different streams or host threads) race; calls ordered on
 * one stream do not.  Nothing in the array needs clearing between calls:
 * each call writes every count and list entry it reads.  Arguments as for
 * mf_integrand. */
#define MF_NOALLOC_MAX_POINTS (1 << 22)
mf_status mf_integrand_noalloc(mf_process* p, const double* u, int64_t n, double* w, void* stream);

/* The same integrand and its derivatives (forward mode) at the same points.
 * The paper computes no derivatives: this extends its event weight (Sec. 2.1)
 * with the derivatives in the top mass and the PDF parameters, by dual
 * numbers through the same steps:
 *   dw: device, [9][n] FP64: d w / d m_t, then d w / d theta_k for
 *       theta = (A_g, a_g, b_g, c_g, d_g, A_u, A_d, A_u~), i.e. pdf_params
 *       entries 0..4, 5, 10, 15.  m_t enters the top momenta, the phase-space
 *       weight, spinors, propagators and (if mu <= 0) the PDF scale.
 * w may be NULL. */
mf_status mf_integrand_grad(mf_process* p, const double* u, int64_t n, double* w, double* dw, void* stream);

/* One VEGAS grid refinement (Lepage 1978) per dimension, on the device:
 * 3-point smoothing of the bin sums of w^2, damped importance
 * r_k = [(1 - d_k/D) / ln(D/d_k)]^alpha, new edges holding equal shares of
 * sum r, linear inside old bins.
 *   edges: device, [ndim][nbins+1] FP64, in/out, strictly increasing.
 *   hist:  device, [ndim][nbins] FP64 sums of w^2 per bin (>= 0).
 *   status: device, one int32 of caller-owned scratch (its content on entry
 *           does not matter; it is cleared by a kernel, not by a memset).
 * A dimension whose histogram is all zero is left unchanged.  MF_ERANGE if
 * the result is not strictly increasing (the input grid is then unchanged
 * for that dimension).  MF_EINVAL for a NULL buffer.  ndim in 1..13, nbins
 * in 1..64.  Allocates nothing; synchronises `stream` before returning. */
mf_status mf_vegas_refine(double* edges, const double* hist, int ndim, int nbins, double alpha, int32_t* status,
                          void* stream);

struct mf_flow;     /* learned proposal, mf_flow.h */
struct mf_result_s; /* mf_result, below */

/* Weighted histograms of observables of the events of a VEGAS integration
 * (the distributions of Sec. 3, here on synthetic inputs).  Observables, in
 * GeV: 0 = transverse momentum of the top quark, 1 = invariant mass of the
 * top pair, 2 = transverse momentum of the hardest final-state gluon (no
 * entries without final gluons).  Uniform bins [lo, hi) per observable;
 * events outside are not binned. */
#define MF_N_OBS 3
typedef struct {
  int32_t nbins;          /* bins per observable, 1..64 */
  double lo[MF_N_OBS];    /* lower edge of each range */
  double hi[MF_N_OBS];    /* upper edge, > lo */
  double* sums;           /* host output [MF_N_OBS][nbins][2]: per bin the sum
                             of w and of w^2 over the events of the counted
                             iterations (those after warmup_iters_discarded) */
  double* sigma;          /* host output [MF_N_OBS][nbins][2], or NULL: per bin
                             the cross section sum w / M (pb) and its Monte
                             Carlo error sqrt((sum w^2 / M - (sum w / M)^2) /
                             (M - 1)), with M = N * (counted iterations) the
                             number of counted events */
} mf_observables;

typedef struct {
  int32_t n_iter;                 /* iterations, >= 1 */
  int64_t n_events;               /* events per iteration, >= 2 */
  double target_rel_err;          /* stop once error/integral <= this; 0 = off */
  int32_t warmup_iters_discarded; /* leading iterations left out of the mean */
  int32_t adapt;                  /* 1: refine the grid after each iteration */
  uint64_t iter_offset;           /* Philox iteration word of the first iteration */
  const double* edges_in;         /* device [ndim][nbins+1] start grid, or NULL = current grid */
  double* edges_out;              /* device [ndim][nbins+1] final grid, or NULL */
  void* stream;                   /* hipStream_t or NULL */
  struct mf_flow* flow;           /* NULL: VEGAS proposal.  Else the flow is the
                                     proposal on the frozen grid (adapt must be
                                     0), see mf_weights */
  double flow_mix;                /* with a flow: the fraction a of uniform
                                     points in the proposal, in [0,1) */
  const struct mf_result_s* prior; /* NULL, or an earlier estimate (integral,
                                     error) that enters the inverse-variance
                                     combination and the target test as one
                                     more iteration */
  const mf_observables* obs;      /* NULL, or histograms to fill (VEGAS
                                     proposal of the single-kernel processes
                                     only: MF_ENOTSUP with a flow, for
                                     g g -> t t~ g g in FP64 and for
                                     g g -> t t~ g g g) */
  double fallback_rel_var;        /* with a flow: 0 = off; > 0 = the per-event
                                     relative variance of the VEGAS proposal
                                     on the same frozen grid.  The first
                                     iteration samples the flow; if its
                                     per-event relative variance
                                     (N - 1) sigma_1^2 / I_1^2 exceeds this
                                     value, that iteration is kept (it is an
                                     unbiased estimate) and every later
                                     iteration samples the VEGAS proposal on
                                     the frozen grid instead (plain VEGAS as
                                     the fallback of the learned proposal) */
} mf_integrate_opts;

typedef struct mf_result_s {
  double integral;          /* inverse-variance weighted mean (pb) */
  double error;             /* its standard error */
  double chi2_dof;          /* chi^2 per degree of freedom of the iterations */
  int32_t n_iter_done;
  int64_t n_events_total;
  int64_t n_nonzero;        /* events with w != 0 */
  int64_t n_nonfinite;      /* events whose weight was not finite (dropped) */
  double seconds;           /* wall time of the call */
  double time_to_target;    /* seconds until error/integral <= target, -1 if never */
  double kernel_seconds;    /* summed device time of the fused per-event kernel,
                               from HIP events recorded around each launch on
                               the call's stream */
  double* iter_integral;    /* host, length >= n_iter, or NULL */
  double* iter_error;       /* host, length >= n_iter, or NULL */
  int32_t fallback_iter;    /* with a flow and fallback_rel_var > 0: index of
                               the first iteration that sampled VEGAS after
                               the fallback, -1 if the flow was kept (also -1
                               without a flow) */
  double flow_rel_var;      /* per-event relative variance of the first flow
                               iteration when the fallback test ran, else -1 */
  double* iter_seconds;     /* host, length >= n_iter, or NULL: with
                               target_rel_err > 0, wall seconds from the start
                               of the call to the end of each iteration (the
                               call waits for every iteration then); else 0 */
} mf_result;

/* VEGAS integration (Lepage 1978) of the integrand: per iteration, events
 * e = 0..n_events-1 draw ndim uniforms from Philox4x64-10 with counter
 * (e, iter_offset + it, call, 0) and key (cfg.seed, 0); the uniforms go
 * through the grid, the weights w = f * Jacobian are reduced (compensated
 * FP64 sums of w and w^2) and binned (w^2 per dimension and bin); the grid
 * is refined on the device.  The handle keeps the final grid.  Events that
 * fail the cuts contribute zero and their matrix element is not evaluated.
 * Under a learned proposal (opts.flow) any non-finite weight is MF_ERANGE
 * (the integrand itself never returns one, so it comes from a broken
 * proposal).  Blocks until the result is on the host. */
mf_status mf_integrate(mf_process* p, const mf_integrate_opts* o, mf_result* r);

/* Per-event weights of one sample with the frozen grid of the handle:
 *  flow == NULL: y from Philox with counter (e, iter, call, 0) and key
 *                (cfg.seed, 0) -- the points of VEGAS iteration `iter` --
 *                and w = f(x(y)) J(y);
 *  flow != NULL: Philox numbers u with key (cfg.seed, 1); with a = flow_mix,
 *                events e < floor(a n) take y = u, the others y = flow
 *                inverse of u (mf_flow.h); w = f(x(y)) J(y) / (a + (1-a) q(y)),
 *                the weight of the mixture of the uniform density and the
 *                flow (unbiased for the fixed split: the two parts sample
 *                their own densities in the proportions a : 1-a).
 *   y_out: device [ndim][n] FP32 copy of y, or NULL
 *   w_out: device [n] FP64 weights (pb)
 * This is how training samples for the flow are drawn and how the weight
 * distributions of the two proposals are compared.  The flow's dimension
 * must equal the process's; flow_mix in [0,1).  Staging buffers of the
 * handle grow to n. */
mf_status mf_weights(mf_process* p, struct mf_flow* flow, double flow_mix, uint64_t iter, int64_t n, float* y_out,
                     double* w_out, void* stream);

/* Statistics of weights (device [n] FP64, n >= 1; they may be negative
 * where the interpolated PDFs dip below zero near x = 1):
 *   out: host [5] = mean, maximum, the q-quantile (the smallest weight with
 *        at least ceil(q n) weights <= it), number of non-zero weights, and
 *        the relative variance per event mean(w^2)/mean(w)^2 - 1 (0 if the
 *        mean is 0), so the Monte Carlo error of the mean of N such weights
 *        is |mean| sqrt(that / N).
 * The quantile is exact (radix selection on order-preserving bit keys).  The
 * unweighting efficiency of a sample is mean / max (or mean / quantile).
 *   work: device scratch owned by the caller, at least
 *         mf_weight_stats_workspace(n) bytes, 8-byte aligned.
 * MF_EINVAL for a NaN weight, q outside (0,1], a NULL or too small
 * workspace.  Allocates nothing.  Synchronous. */
mf_status mf_weight_stats(const double* w, int64_t n, double q, double* out, void* work, int64_t work_bytes,
                          void* stream);
/* Bytes of device scratch mf_weight_stats needs for n weights (n >= 1). */
int64_t mf_weight_stats_workspace(int64_t n);

/* Vector-Jacobian product of per-event derivatives with an upstream
 * gradient (the backward step of an autograd function over
 * mf_integrand_grad):
 *   dw:  device [k][n] FP64 (e.g. the dw of mf_integrand_grad, k = 9)
 *   g:   device [n] FP64 upstream gradient of the per-event weights
 *   out: device [k] FP64, out[j] = sum_e dw[j][e] g[e] (ordered, reproducible)
 *   work: device scratch owned by the caller, at least mf_vjp_workspace(k, n)
 *         bytes, 8-byte aligned, not read before it is written.
 * k in 1..64, n >= 1; MF_EINVAL otherwise or for a NULL or too small
 * workspace.  Allocates nothing; asynchronous on `stream`. */
mf_status mf_vjp(const double* dw, int32_t k, const double* g, int64_t n, double* out, void* work, int64_t work_bytes,
                 void* stream);
/* Bytes of device scratch mf_vjp needs for k rows of n events. */
int64_t mf_vjp_workspace(int32_t k, int64_t n);

/* Pathwise Monte Carlo estimate of sigma and its parameter derivatives (an
 * extension: the paper integrates sigma only, Sec. 2.1 and 3) with
 * a frozen grid (the current grid of the handle, or o->edges_in): events as
 * in mf_integrate with iteration word o->iter_offset, o->n_events events.
 *   out:  host [10]: sigma, d sigma/d m_t, d sigma / d theta_k (k = 0..7)
 *   err:  host [10]: their Monte Carlo standard errors
 * Only n_events, iter_offset, edges_in and stream of o are used. */
mf_status mf_grad(mf_process* p, const mf_integrate_opts* o, double* out, double* err);

#ifdef __cplusplus
}
#endif

#endif /* MF_H */
