// g g -> t t~ g g with the colour sum on the matrix cores (HIP, gfx950).
//
// The 24 colour-ordered partial amplitudes of each helicity state are
// streamed out of the amplitude kernel instead of being contracted with the
// colour matrix in registers, and the colour quadratic form
// |M|^2 = sum_states Re(A^dagger C A) runs as a batched product Z = C A on
// the matrix cores followed by the dot product A . Z:
//
//  1. st::k_st_select: kinematics, cuts and PDFs of every point; the indices
//     of the points that pass are compacted into a list.
//  2. k_s2_amp<R>: per passing event (one lane each), the partial amplitudes
//     of HGP gluon polarisation states (both antitop and both top
//     helicities) from the generated per-ordering Berends-Giele code
//     (amp_gg_m4_store, the same steps as the in-register form), written to
//     a buffer laid out as [slice][ordering / 4][event][ordering % 4]; the
//     per-event propagator factors, polarisation vectors, momenta and
//     antitop spinors sit in per-lane LDS tables, so that nothing per event
//     but the top spinors stays live in registers across the orderings.
//  3. k_s2_colour<R>: per tile of 32 events and per slice, Z = C A with the
//     exact 24 x 24 colour matrix (numerators over 54) padded to 32, on
//     v_mfma_f32_16x16x4_f32 (R = float) or v_mfma_f64_16x16x4_f64
//     (R = double); the operand values loaded for the product are the ones
//     the dot product needs, so each amplitude is read once.
//
// This is the event weight of Sec. 2.1 with the colour-ordered amplitudes
// and colour matrix of Sec. 2.2 (the helicity loop and the aggregation over
// colour flows), as three kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "amp.h"
#include "gen/amps_gg_m4.h"
#include "launch.h"
#include "pipeline.h"
#include "staged.h"

namespace mf {
namespace s2 {

constexpr int NG = 2;
constexpr int M = NG + 2;
constexpr int NF = AMPS_M4_NF;       // 24 orderings
constexpr int NQ = AMPS_M4_NQ;       // 6 groups of four
constexpr int HG = AMPS_M4_HG;       // 16 gluon polarisation states
constexpr int AW = 64;               // amplitude kernel block: one wave (LDS tables per lane)
constexpr int CT = 32;               // events per colour tile (two 16-column MFMA blocks)
constexpr int CBLOCK = 256;          // colour kernel block: 4 waves, each a quarter of the slices
constexpr int CMAX_BLOCKS = 1024;
constexpr int64_t NCMAX = 65536;     // passing events per chunk (1024 amplitude waves)
// gluon polarisation states per pass: 8 slices each (2 antitop x 2 top x re/im)
template <class R> constexpr int HGP = std::is_same<R, float>::value ? 4 : 2;
template <class R> constexpr int SLICES = 8 * HGP<R>;

struct Ws {
  int64_t cap_n = 0;  // points: idx, wpre
  int64_t ld = 0;     // chunk columns of the amplitude buffer (multiple of AW)
  int* d_idx = nullptr;
  int* d_count = nullptr;
  double* d_wpre = nullptr;
  double* d_me = nullptr;  // [ld] colour-summed |M|^2 numerators of the chunk
  void* d_amp = nullptr;   // [SLICES][NQ][ld][4] amplitude type
};

// Partial amplitudes of gluon states hg0 .. hg0 + HGP - 1 for the passing
// events idx[0 .. nc-1] of this chunk, written to
//   amp[((slice * NQ + ordering / 4) * ld + j) * 4 + ordering % 4]
// (j = the event's column).  Lanes past nc recompute the chunk's last event
// into their own columns below ld, which are never read as results.
template <class R>
__global__ void __launch_bounds__(AW) k_s2_amp(DevCfg c, const double* __restrict__ u, int64_t n,
                                               const int* __restrict__ idx, int64_t nc, int hg0,
                                               R* __restrict__ amp, int64_t ld) {
  __shared__ R gtab[16][AW];      // -1 / P_S^2 for gluon subsets S (>= 2 gluons)
  __shared__ R qtab[16][AW];      // -1 / ((p_tb + P_S)^2 - m_t^2) for S != all
  __shared__ V4<R> etab[8][AW];   // polarisation p of gluon i at 2 i + p
  __shared__ V4<R> ktab[4][AW];   // gluon momenta
  __shared__ Sp<R> vtab[2][AW];   // v(antitop) for both helicities
  const int lane = threadIdx.x;
  const int64_t j = (int64_t)blockIdx.x * AW + lane;
  const int64_t e = idx[j < nc ? j : nc - 1];
  double x[MAXD];
#pragma unroll
  for (int k = 0; k < MAXD; ++k)
    if (k < c.ndim) x[k] = u[(int64_t)k * n + e];
  double shat_k, wps;
  V4<double> gl[NG], top, atop;
  (void)st::kinematics<NG>(c, x, shat_k, gl, top, atop, wps);
  // external states as in me_gg: incoming beams as outgoing momenta with
  // fixed linear polarisations, final gluons with lin_pols
  const double E = 0.5 * sqrt(shat_k);
  V4<double> K[M];
  K[0] = V4<double>{-E, 0.0, 0.0, -E};
  K[1] = V4<double>{-E, 0.0, 0.0, E};
  K[2] = gl[0];
  K[3] = gl[1];
  const R z = R(0.0), o = R(1.0);
  etab[0][lane] = V4<R>{z, o, z, z};
  etab[1][lane] = V4<R>{z, z, o, z};
  etab[2][lane] = V4<R>{z, o, z, z};
  etab[3][lane] = V4<R>{z, z, o, z};
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    V4<R> ep[2];
    lin_pols(cvt4<R>(K[2 + i]), ep);
    etab[4 + 2 * i][lane] = ep[0];
    etab[5 + 2 * i][lane] = ep[1];
  }
  for (int S = 1; S < 16; ++S) {
    V4<double> P{0.0, 0.0, 0.0, 0.0};
    bool firstk = true;
#pragma unroll
    for (int i = 0; i < M; ++i)
      if ((S >> i) & 1) {
        P = firstk ? K[i] : P + K[i];
        firstk = false;
      }
    gtab[S][lane] = __popc(S) >= 2 ? cvt<R>(-1.0 / mdot(P, P)) : R(0.0);
    qtab[S][lane] = S != 15 ? cvt<R>(-1.0 / (2.0 * mdot(atop, P) + mdot(P, P))) : R(0.0);
  }
#pragma unroll
  for (int i = 0; i < M; ++i) ktab[i][lane] = cvt4<R>(K[i]);
  const R MT = cvt<R>(c.mt);
  const V4<R> t = cvt4<R>(top), PB = cvt4<R>(atop);
  const Sp<R> UB[2] = {ubar_spinor(t, MT, -1), ubar_spinor(t, MT, 1)};
  vtab[0][lane] = v_spinor(PB, MT, -1);
  vtab[1][lane] = v_spinor(PB, MT, 1);
  // each lane reads only its own column of the tables: no barrier needed
  const int64_t sstride = (int64_t)NQ * ld * 4;
  amp_gg_m4_store<R, AW>(&gtab[0][lane], &qtab[0][lane], &etab[0][lane], &ktab[0][lane], &vtab[0][lane], UB, PB,
                         MT, hg0, HGP<R>, amp + j * 4, sstride, 4 * ld);
}

template <class R> struct Mfma;
template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 step(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 step(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// Colour index that lane group g (= lane / 16) supplies at step (s, r) of a
// 16 x 16 x 4 product, chosen so that the four indices a lane supplies for
// block s = rb are the four rows of Z it receives: the FP32 product returns
// rows 4 g + i to lane group g, the FP64 product rows g + 4 i (i = 0..3).
template <class R> __device__ __forceinline__ constexpr int kidx(int s, int g, int r) {
  return std::is_same<R, float>::value ? 16 * s + 4 * g + r : 16 * s + g + 4 * r;
}

// Colour sum of one pass over the nsl slices (a multiple of 4) of the buffer
// for the nc events of the chunk.  C in LDS in A-operand order: entry
// ((rb * 2 + s) * 64 + l) * 4 + r holds C[16 rb + l % 16][kidx(s, l / 16, r)]
// (zero beyond the 24 orderings).  For the step (s, r) lane l supplies that
// entry and B[kidx(s, l / 16, r)][event l % 16] (zero beyond the 24
// orderings), so the four lane groups cover colour indices 16 s .. 16 s + 15
// over the four r; the result lane l holds Z[kidx(rb, l / 16, i)][event
// l % 16] in its element i, whose matching amplitudes are the B values the
// lane loaded for s = rb.  first: the pass overwrites me[]; last: it also
// writes the weights.
template <class R>
__global__ void __launch_bounds__(CBLOCK) k_s2_colour(const R* __restrict__ amp, int64_t ld, int64_t nc, int nsl,
                                                      int first, int last, double* __restrict__ me,
                                                      const int* __restrict__ idx, const double* __restrict__ wpre,
                                                      double* __restrict__ w, double inv_den) {
  typedef typename Mfma<R>::v4 v4;
  __shared__ R cs[2 * 2 * 64 * 4];
  __shared__ double part[CBLOCK / 64][CT];
  for (int i = threadIdx.x; i < 2 * 2 * 64 * 4; i += CBLOCK) {
    const int r = i & 3, l = (i >> 2) & 63, s = (i >> 8) & 1, rb = i >> 9;
    const int row = 16 * rb + (l & 15), col = kidx<R>(s, l >> 4, r);
    cs[i] = (row < NF && col < NF) ? R(AMPS_M4_COLOUR[row * NF + col]) : R(0.0);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, c16 = lane & 15;
  const int64_t ntile = (nc + CT - 1) / CT;
  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int64_t c0 = tile * CT;
    double sum[2] = {0.0, 0.0};
#pragma unroll 1
    for (int sl = wave * (nsl / 4); sl < (wave + 1) * (nsl / 4); ++sl) {
      const R* base = amp + (int64_t)sl * NQ * ld * 4;
      v4 bv[2][2];
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          const int64_t col = c0 + 16 * cb + c16;
          if constexpr (std::is_same<R, float>::value) {
            // the four orderings 16 s + 4 g + r are one group of four: one load
            const int q = 4 * s + g;
            bv[s][cb] = q < NQ ? *reinterpret_cast<const v4*>(base + ((int64_t)q * ld + col) * 4)
                               : v4{R(0.0), R(0.0), R(0.0), R(0.0)};
          } else {
            // orderings 16 s + g + 4 r: element g of the groups 4 s + r
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int q = 4 * s + r;
              bv[s][cb][r] = q < NQ ? base[((int64_t)q * ld + col) * 4 + g] : R(0.0);
            }
          }
        }
      R acc[2] = {R(0.0), R(0.0)};
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        v4 zz[2] = {v4{R(0.0), R(0.0), R(0.0), R(0.0)}, v4{R(0.0), R(0.0), R(0.0), R(0.0)}};
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const v4 a = *reinterpret_cast<const v4*>(&cs[((rb * 2 + s) * 64 + lane) * 4]);
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) zz[cb] = Mfma<R>::step(a[r], bv[s][cb][r], zz[cb]);
        }
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[cb] = fma(zz[cb][i], bv[rb][cb][i], acc[cb]);
      }
      sum[0] += (double)acc[0];
      sum[1] += (double)acc[1];
    }
    // the four lane groups hold disjoint rows of the same events
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
      sum[cb] += __shfl_xor(sum[cb], 16);
      sum[cb] += __shfl_xor(sum[cb], 32);
    }
    if (g == 0) {
      part[wave][c16] = sum[0];
      part[wave][16 + c16] = sum[1];
    }
    __syncthreads();
    if (threadIdx.x < CT) {
      const int64_t col = c0 + threadIdx.x;
      if (col < nc) {
        double v = part[0][threadIdx.x];
#pragma unroll
        for (int q = 1; q < CBLOCK / 64; ++q) v += part[q][threadIdx.x];
        if (!first) v += me[col];
        me[col] = v;
        if (last) {
          const int e = idx[col];
          const double we = wpre[e] * (v * inv_den);
          w[e] = isfinite(we) ? we : 0.0;
        }
      }
    }
    __syncthreads();
  }
}

inline void ws_free(void* p) {
  Ws* ws = static_cast<Ws*>(p);
  if (!ws) return;
  (void)hipFree(ws->d_idx);
  (void)hipFree(ws->d_count);
  (void)hipFree(ws->d_wpre);
  (void)hipFree(ws->d_me);
  (void)hipFree(ws->d_amp);
  delete ws;
}

#define S2_TRY(expr)                  \
  do {                                \
    hipError_t e_ = (expr);           \
    if (e_ != hipSuccess) return e_;  \
  } while (0)

// The integrand at n points: selection, then per chunk of passing events
// the amplitude and colour kernels in passes over the gluon polarisation
// states.  Synchronises the stream once (to read the number of passing
// events).  The workspace grows on demand and belongs to the process handle.
template <class R>
hipError_t integrand(const DevCfg& c, const double* u, int64_t n, double* w, void** wsp, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  Ws* ws = static_cast<Ws*>(*wsp);
  if (!ws) {
    ws = new Ws();
    *wsp = ws;
    S2_TRY(hipMalloc(&ws->d_count, sizeof(int)));
  }
  if (ws->cap_n < n) {
    S2_TRY(hipStreamSynchronize(s));
    (void)hipFree(ws->d_idx);
    (void)hipFree(ws->d_wpre);
    ws->d_idx = nullptr;
    ws->d_wpre = nullptr;
    ws->cap_n = 0;
    S2_TRY(hipMalloc(&ws->d_idx, sizeof(int) * n));
    S2_TRY(hipMalloc(&ws->d_wpre, sizeof(double) * n));
    ws->cap_n = n;
  }
  hipLaunchKernelGGL(st::k_st_zero, dim3(1), dim3(1), 0, s, ws->d_count);
  hipLaunchKernelGGL(st::k_st_select<NG>, dim3((unsigned)((n + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, s, c, u, n, w,
                     ws->d_wpre, ws->d_idx, ws->d_count);
  S2_TRY(hipGetLastError());
  int count = 0;
  S2_TRY(hipMemcpyAsync(&count, ws->d_count, sizeof(int), hipMemcpyDeviceToHost, s));
  S2_TRY(hipStreamSynchronize(s));
  if (count <= 0) return hipSuccess;
  // chunk width: the passing events, up to NCMAX, rounded to the amplitude block
  int64_t want = count < NCMAX ? (int64_t)count : NCMAX;
  want = (want + AW - 1) / AW * AW;
  if (ws->ld < want) {
    S2_TRY(hipStreamSynchronize(s));
    (void)hipFree(ws->d_amp);
    (void)hipFree(ws->d_me);
    ws->d_amp = nullptr;
    ws->d_me = nullptr;
    ws->ld = 0;
    S2_TRY(hipMalloc(&ws->d_amp, sizeof(R) * (size_t)SLICES<R> * NQ * (size_t)want * 4));
    S2_TRY(hipMalloc(&ws->d_me, sizeof(double) * want));
    ws->ld = want;
  }
  const int64_t ld = ws->ld;
  R* amp = static_cast<R*>(ws->d_amp);
  constexpr int NPASS = HG / HGP<R>;
  const double inv_den = 1.0 / AMPS_M4_COLOUR_DEN;
  for (int64_t c0 = 0; c0 < count; c0 += ld) {
    const int64_t nc = (count - c0) < ld ? (count - c0) : ld;
    const int* idx = ws->d_idx + c0;
    const unsigned ablk = (unsigned)((nc + AW - 1) / AW);
    const int64_t ntile = (nc + CT - 1) / CT;
    const unsigned cblk = (unsigned)(ntile < CMAX_BLOCKS ? ntile : CMAX_BLOCKS);
    for (int pass = 0; pass < NPASS; ++pass) {
      hipLaunchKernelGGL((k_s2_amp<R>), dim3(ablk), dim3(AW), 0, s, c, u, n, idx, nc, pass * HGP<R>, amp, ld);
      hipLaunchKernelGGL((k_s2_colour<R>), dim3(cblk), dim3(CBLOCK), 0, s, amp, ld, nc, SLICES<R>,
                         pass == 0 ? 1 : 0, pass == NPASS - 1 ? 1 : 0, ws->d_me, idx, ws->d_wpre, w, inv_den);
    }
    S2_TRY(hipGetLastError());
  }
  return hipSuccess;
}

#undef S2_TRY

template <class R>
Launchers launchers() {
  Launchers L;
  L.fused = false;
  L.integrand = nullptr;
  L.vegas = nullptr;
  L.integrand_grad = nullptr;
  L.grad_vegas = nullptr;
  L.observables = nullptr;
  L.integrand_ws = integrand<R>;
  L.ws_free = ws_free;
  return L;
}

}  // namespace s2
}  // namespace mf
