// Kernel instance: gg3_f32 (g g -> t t~ g g g, FP32 amplitudes, FP64
// kinematics, PDFs and weights), evaluated by the staged kernels of gg3.h.
#include "gg3.h"

namespace mf {
namespace g3 {
namespace {

void ws_free(void* p) {
  Ws* ws = static_cast<Ws*>(p);
  if (!ws) return;
  (void)hipFree(ws->d_idx);
  (void)hipFree(ws->d_count);
  (void)hipFree(ws->d_wpre);
  (void)hipFree(ws->d_me);
  (void)hipFree(ws->d_amp);
  delete ws;
}

#define G3_TRY(expr)                  \
  do {                                \
    hipError_t e_ = (expr);           \
    if (e_ != hipSuccess) return e_;  \
  } while (0)

hipError_t integrand(const DevCfg& c, const double* u, int64_t n, double* w, void** wsp, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  Ws* ws = static_cast<Ws*>(*wsp);
  if (!ws) {
    ws = new Ws();
    *wsp = ws;
    G3_TRY(hipMalloc(&ws->d_count, sizeof(int)));
  }
  if (ws->cap_n < n) {
    G3_TRY(hipStreamSynchronize(s));
    (void)hipFree(ws->d_idx);
    (void)hipFree(ws->d_wpre);
    ws->d_idx = nullptr;
    ws->d_wpre = nullptr;
    ws->cap_n = 0;
    G3_TRY(hipMalloc(&ws->d_idx, sizeof(int) * n));
    G3_TRY(hipMalloc(&ws->d_wpre, sizeof(double) * n));
    ws->cap_n = n;
  }
  hipLaunchKernelGGL(st::k_st_zero, dim3(1), dim3(1), 0, s, ws->d_count);
  hipLaunchKernelGGL(st::k_st_select<NG>, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, c, u, n, w,
                     ws->d_wpre, ws->d_idx, ws->d_count);
  G3_TRY(hipGetLastError());
  int count = 0;
  G3_TRY(hipMemcpyAsync(&count, ws->d_count, sizeof(int), hipMemcpyDeviceToHost, s));
  G3_TRY(hipStreamSynchronize(s));
  if (count <= 0) return hipSuccess;
  // chunk width: the passing events, up to NCMAX, rounded to the amplitude block
  int64_t want = count < NCMAX ? (int64_t)count : NCMAX;
  want = (want + AWAVE - 1) / AWAVE * AWAVE;
  if (ws->ld < want) {
    (void)hipFree(ws->d_amp);
    (void)hipFree(ws->d_me);
    ws->d_amp = nullptr;
    ws->d_me = nullptr;
    ws->ld = 0;
    const size_t bytes = sizeof(float) * (size_t)SLICES * NQ * (size_t)want * 4;
    G3_TRY(hipMalloc(&ws->d_amp, bytes));
    G3_TRY(hipMalloc(&ws->d_me, sizeof(double) * want));
    ws->ld = want;
    ws->amp_bytes = bytes;
  }
  const int64_t ld = ws->ld;
  float* amp = static_cast<float*>(ws->d_amp);
  // all states in passes of SP, or one state per point in a single pass
  const bool own = c.helicity != 0;
  const int NPASS = own ? 1 : STATES / SP, ns = own ? 1 : SP, nsl = 4 * ns;
  const double inv_den = (c.helicity == 1 ? (double)STATES : 1.0) / AMP_M5_COLOUR_DEN;
  for (int64_t c0 = 0; c0 < count; c0 += ld) {
    const int64_t nc = (count - c0) < ld ? (count - c0) : ld;
    const int* idx = ws->d_idx + c0;
    const unsigned ablk = (unsigned)((nc + AWAVE - 1) / AWAVE);
    const int64_t ntile = (nc + CT - 1) / CT;
    const unsigned cblk = (unsigned)(ntile < CMAX_BLOCKS ? ntile : CMAX_BLOCKS);
    for (int pass = 0; pass < NPASS; ++pass) {
      hipLaunchKernelGGL((k_g3_amp<float>), dim3(ablk), dim3(AWAVE), 0, s, c, u, n, idx, nc, pass * SP, ns, amp, ld);
      hipLaunchKernelGGL(k_g3_colour, dim3(cblk), dim3(CBLOCK), 0, s, amp, ld, nc, nsl, pass == 0 ? 1 : 0,
                         pass == NPASS - 1 ? 1 : 0, ws->d_me, idx, ws->d_wpre, w, inv_den);
    }
    G3_TRY(hipGetLastError());
  }
  return hipSuccess;
}

}  // namespace
}  // namespace g3

Launchers launchers_gg3_f32() {
  Launchers L;
  L.fused = false;
  L.integrand = nullptr;
  L.vegas = nullptr;
  L.integrand_grad = nullptr;
  L.grad_vegas = nullptr;
  L.observables = nullptr;
  L.integrand_ws = g3::integrand;
  L.ws_free = g3::ws_free;
  return L;
}

}  // namespace mf
