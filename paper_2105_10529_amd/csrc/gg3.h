// g g -> t t~ g g g: staged evaluation of the integrand (HIP, gfx950).
//
// With 120 colour orderings and 128 helicity states per event the partial
// amplitudes of one event do not fit in registers next to the colour
// quadratic form, so the evaluation of a batch of points is split:
//
//  1. st::k_st_select (staged.h): kinematics, cuts and PDFs of every point (FP64); the
//     weight without |M|^2 is kept, and the indices of the events that pass
//     the cuts are compacted into a list, so the amplitudes run on passing
//     events only.
//  2. k_g3_amp: per passing event (one lane each), the colour-ordered partial
//     amplitudes of a group of polarisation states (generated per-ordering
//     Berends-Giele code, amp_gg_m5), streamed to an HBM buffer laid out as
//     [slice][ordering / 4][event][ordering % 4].
//  3. k_g3_colour: the colour sum |M|^2 = sum_states Re(A^dagger C A) with
//     the exact 120 x 120 colour matrix on the matrix cores
//     (v_mfma_f32_16x16x4_f32): per slice, Z = C A for a tile of 32 events,
//     then the dot product A . Z in the epilogue; the operand values loaded
//     for the product are the ones the dot product needs, so each amplitude
//     is read once.
//
// This is the event weight of Sec. 2.1 (phase space -> matrix element) with
// the colour-ordered amplitudes and colour matrix of Sec. 2.2, evaluated in
// the three-kernel order above; the result of each event does not depend on
// the lane or the position in the compacted list that evaluates it.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "amp.h"
#include "gen/amp_gg_m5.h"
#include "launch.h"
#include "pipeline.h"
#include "staged.h"

namespace mf {
namespace g3 {

constexpr int NG = 3;
constexpr int NF = AMP_M5_NF;          // 120 orderings
constexpr int NQ = AMP_M5_NQ;          // 32 groups of four (padded to 128)
constexpr int STATES = AMP_M5_STATES;  // 64 = 2 antitop helicities x 2^5 gluon polarisations
constexpr int SP = 8;                  // states per amplitude pass
constexpr int SLICES = SP * 4;         // (state, top helicity, re/im) per pass
constexpr int AWAVE = 64;              // amplitude kernel block: one wave (LDS tables per wave)
constexpr int CT = 32;                 // events per colour tile (two 16-column MFMA blocks)
constexpr int CBLOCK = 256;            // colour kernel block: 4 waves x 8 slices
constexpr int CMAX_BLOCKS = 512;       // two 65-KB-LDS blocks per CU
constexpr int64_t NCMAX = 131072;      // passing events per chunk (fills 256 CUs x 2 waves x 4 SIMDs)
// FP64 amplitudes: half the chunk (the same buffer size)
template <class R> constexpr int64_t NCMAX_R = std::is_same<R, float>::value ? NCMAX : NCMAX / 2;

// Workspace owned by the process handle (grown on demand, freed with it).
struct Ws {
  int64_t cap_n = 0;  // points: idx, wpre
  int64_t ld = 0;     // chunk columns of the amplitude buffer (multiple of AWAVE)
  size_t amp_bytes = 0;
  int* d_idx = nullptr;
  int* d_count = nullptr;
  double* d_wpre = nullptr;
  double* d_me = nullptr;  // [ld] colour-summed |M|^2 numerators of the chunk
  void* d_amp = nullptr;   // [SLICES][NQ][ld][4] amplitude type
};

using st::kinematics;

// One colour-ordered partial amplitude for both top helicities: the gluon
// currents J(a..b) of every contiguous range of positions (Berends-Giele,
// three- and four-gluon vertices; gluon_stage), then the top-line spinor
// currents of every suffix closed by the top propagator and the final
// contraction with ubar(top) (spinor_stage; the same steps, in the same order
// of terms, as the per-ordering amplitudes of the smaller processes).  The
// gluon currents do not depend on the antitop helicity, so one gluon stage
// serves the spinor stages of both.  J[a][a], P[a][a]: external current and
// momentum at position a; g[r]: propagator factor of range r in AMP_M5_RANGE
// order; iq[j]: factor of the suffix starting at position j + 1; S[5]: the
// antitop spinor.  In two stages each: SUFFIX = true computes what depends on
// positions 2..4 only (the currents of the ranges inside them and the spinor
// currents S[2..4]), which two orderings that differ by the swap of their
// first two gluons share; SUFFIX = false completes the ordering from them.
template <class R, bool SUFFIX>
__device__ __forceinline__ void gluon_stage(V4<R> (&J)[5][5], V4<R> (&P)[5][5], const R (&g)[10]) {
  int r = 0;  // range index in AMP_M5_RANGE order: by length, then start
#pragma unroll
  for (int len = 2; len <= 5; ++len)
#pragma unroll
  for (int a = 0; a + len <= 5; ++a, ++r) {
    if (SUFFIX != (a >= 2)) continue;
    const int b = a + len - 1;
    P[a][b] = P[a][b - 1] + P[b][b];
    // the vertices accumulate into one current (fused multiply-add chains)
    V4<R> t = v3(J[a][a], J[a + 1][b], P[a][a], P[a + 1][b]);
#pragma unroll
    for (int j = a + 1; j < b; ++j) t = v3_acc(J[a][j], J[j + 1][b], P[a][j], P[j + 1][b], t);
#pragma unroll
    for (int j = a; j < b - 1; ++j)
#pragma unroll
      for (int l = j + 1; l < b; ++l) t = w4_sub(J[a][j], J[j + 1][l], J[l + 1][b], t);
    J[a][b] = g[r] * t;
  }
}

template <class R, bool SUFFIX>
__device__ __forceinline__ void spinor_stage(const V4<R> (&J)[5][5], const V4<R> (&P)[5][5], Sp<R> (&S)[6],
                                             const R (&iq)[4], const V4<R>& pb, R MT, const Sp<R>* UB, C2<R>& A0,
                                             C2<R>& A1) {
#pragma unroll
  for (int a = 4; a >= 1; --a) {
    if (SUFFIX != (a >= 2)) continue;
    Sp<R> acc = slash(J[a][a], S[a + 1]);
#pragma unroll
    for (int j = a + 1; j < 5; ++j) acc = slash_acc(J[a][j], S[j + 1], acc);
    S[a] = prop_neg(pb + P[a][4], MT, iq[a - 1], acc);
  }
  if (!SUFFIX) {
    Sp<R> F = slash(J[0][0], S[1]);
#pragma unroll
    for (int j = 1; j < 5; ++j) F = slash_acc(J[0][j], S[j + 1], F);
    A0 = ubar_dot(UB[0], F);
    A1 = ubar_dot(UB[1], F);
  }
}

// Partial amplitudes of states s0 .. s0 + ns - 1 for the passing events
// idx[0 .. nc-1] of this chunk, written to
//   amp[((slice * NQ + ordering / 4) * ld + j) * 4 + ordering % 4]
// with slice = ((state - s0) * 2 + top helicity) * 2 + (0: re, 1: im) and
// j the event's column (orderings 120..127 are written as zeros).  Lanes
// past nc recompute the last event into columns below ld, never read as
// results.  The propagator factors of every gluon subset are formed in FP64
// from the FP64 momenta and kept per lane in LDS, indexed by subset.
// With c.helicity != 0 each lane evaluates one state k of its own (ns = 1;
// antitop helicity k / 32, gluon polarisation state k % 32): drawn by Philox
// from the point's first two coordinates (mode 1) or the fixed state
// helicity - 2; the ordering loop stays wave-uniform.  In the summed mode
// (ns even) pass state s stands for gluon polarisation state s / 2 and
// antitop helicity s % 2, so that both antitop helicities of a gluon state
// are evaluated together from one set of gluon currents.
static_assert(SP % 2 == 0, "summed passes hold both antitop helicities of each gluon state");
template <class R>
__global__ void __launch_bounds__(AWAVE) k_g3_amp(DevCfg c, const double* __restrict__ u, int64_t n,
                                                  const int* __restrict__ idx, int64_t nc, int s0, int ns,
                                                  R* __restrict__ amp, int64_t ld) {
  // Per-lane tables (each lane reads only its own column, so no barriers):
  __shared__ R gtab[32][AWAVE];        // -1 / P_S^2 for gluon subsets S (>= 2 gluons)
  __shared__ R qtab[32][AWAVE];        // -1 / ((p_tb + P_S)^2 - m_t^2) for S != all
  __shared__ V4<R> etab[10][AWAVE];    // polarisation vectors: gluon i, polarisation p at 2 i + p
  __shared__ V4<R> ktab[5][AWAVE];     // gluon momenta in the amplitude type
  __shared__ Sp<R> vtab[2][AWAVE];     // v(antitop) for both helicities
  const int lane = threadIdx.x;
  const int64_t j = (int64_t)blockIdx.x * AWAVE + lane;
  const int64_t e = idx[j < nc ? j : nc - 1];
  double x[MAXD];
#pragma unroll
  for (int k = 0; k < MAXD; ++k)
    if (k < c.ndim) x[k] = u[(int64_t)k * n + e];
  double shat_k, wps;
  V4<double> gl[NG], top, atop;
  (void)kinematics<NG>(c, x, shat_k, gl, top, atop, wps);
  // external states as in me_gg: incoming beams as outgoing momenta with
  // fixed linear polarisations, final gluons with lin_pols, top spinors of
  // both helicities
  const double E = 0.5 * sqrt(shat_k);
  V4<double> K[NG + 2];
  V4<R> Ep[NG + 2][2];
  K[0] = V4<double>{-E, 0.0, 0.0, -E};
  K[1] = V4<double>{-E, 0.0, 0.0, E};
  const R z = R(0.0), o = R(1.0);
  Ep[0][0] = V4<R>{z, o, z, z};
  Ep[0][1] = V4<R>{z, z, o, z};
  Ep[1][0] = V4<R>{z, o, z, z};
  Ep[1][1] = V4<R>{z, z, o, z};
#pragma unroll
  for (int i = 0; i < NG; ++i) {
    K[2 + i] = gl[i];
    lin_pols(cvt4<R>(K[2 + i]), Ep[2 + i]);
  }
  for (int S = 1; S < 32; ++S) {
    V4<double> P{0.0, 0.0, 0.0, 0.0};
    bool firstk = true;
#pragma unroll
    for (int i = 0; i < 5; ++i)
      if ((S >> i) & 1) {
        P = firstk ? K[i] : P + K[i];
        firstk = false;
      }
    gtab[S][lane] = __popc(S) >= 2 ? cvt<R>(-1.0 / mdot(P, P)) : R(0.0);
    qtab[S][lane] = S != 31 ? cvt<R>(-1.0 / (2.0 * mdot(atop, P) + mdot(P, P))) : R(0.0);
  }
  const R MT = cvt<R>(c.mt);
  const V4<R> t = cvt4<R>(top), PB = cvt4<R>(atop);
  const Sp<R> UB[2] = {ubar_spinor(t, MT, -1), ubar_spinor(t, MT, 1)};
  vtab[0][lane] = v_spinor(PB, MT, -1);
  vtab[1][lane] = v_spinor(PB, MT, 1);
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    ktab[i][lane] = cvt4<R>(K[i]);
    etab[2 * i][lane] = Ep[i][0];
    etab[2 * i + 1][lane] = Ep[i][1];
  }
  const int64_t sstride = (int64_t)NQ * ld * 4;
  R* out = amp + j * 4;
  int own = -1;  // this lane's state when states are sampled or fixed
  if (c.helicity == 1) {
    const U4 r = philox4x64_10((uint64_t)__double_as_longlong(x[0]), (uint64_t)__double_as_longlong(x[1]), 0, 0,
                               c.seed, 5);
    own = (int)(r.x0 >> 58);
  } else if (c.helicity >= 2) {
    own = c.helicity - 2;
  }
  // The 120 orderings of gluon polarisation state hg for NH antitop
  // helicities (ht0 .. ht0 + NH - 1), written at slots 0 .. NH - 1 of o4.
  auto orderings = [&](auto nh, int hg, int ht0, R* o4) {
    constexpr int NH = decltype(nh)::value;
#pragma unroll 1
    for (int pr = 0; pr < AMP_M5_NPAIR; ++pr) {
      V4<R> J[5][5], P[5][5];
      Sp<R> S[NH][6];
      R gr[10], iq[4];
      C2<R> a0, a1;
      {
        // positions 2..4 hold the same gluons in both orderings of the pair
        const int k = AMP_M5_PAIR[pr][0];
#pragma unroll
        for (int i = 2; i < 5; ++i) {
          const int sg = AMP_M5_SIGMA[k][i];
          J[i][i] = etab[2 * sg + ((hg >> (4 - sg)) & 1)][lane];
          P[i][i] = ktab[sg][lane];
        }
        gr[2] = gtab[AMP_M5_GMASK[k][2]][lane];
        gr[3] = gtab[AMP_M5_GMASK[k][3]][lane];
        gr[6] = gtab[AMP_M5_GMASK[k][6]][lane];
#pragma unroll
        for (int j = 1; j < 4; ++j) iq[j] = qtab[AMP_M5_QMASK[k][j]][lane];
        gluon_stage<R, true>(J, P, gr);
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          S[h][5] = vtab[ht0 + h][lane];
          spinor_stage<R, true>(J, P, S[h], iq, PB, MT, UB, a0, a1);
        }
      }
#pragma unroll
      for (int o = 0; o < 2; ++o) {
        const int k = AMP_M5_PAIR[pr][o];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const int sg = AMP_M5_SIGMA[k][i];
          J[i][i] = etab[2 * sg + ((hg >> (4 - sg)) & 1)][lane];
          P[i][i] = ktab[sg][lane];
        }
        gr[0] = gtab[AMP_M5_GMASK[k][0]][lane];
        gr[1] = gtab[AMP_M5_GMASK[k][1]][lane];
        gr[4] = gtab[AMP_M5_GMASK[k][4]][lane];
        gr[5] = gtab[AMP_M5_GMASK[k][5]][lane];
#pragma unroll
        for (int r = 7; r < 10; ++r) gr[r] = gtab[AMP_M5_GMASK[k][r]][lane];
        iq[0] = qtab[AMP_M5_QMASK[k][0]][lane];
        gluon_stage<R, false>(J, P, gr);
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          spinor_stage<R, false>(J, P, S[h], iq, PB, MT, UB, a0, a1);
          R* p = o4 + (int64_t)(h * 4) * sstride + (int64_t)(k >> 2) * ld * 4 + (k & 3);
          p[0] = a0.re;
          p[sstride] = a0.im;
          p[2 * sstride] = a1.re;
          p[3 * sstride] = a1.im;
        }
      }
    }
    // zero padding of the orderings NF .. 4 NQ - 1
#pragma unroll 1
    for (int k = NF; k < 4 * NQ; ++k) {
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        R* p = o4 + (int64_t)(h * 4) * sstride + (int64_t)(k >> 2) * ld * 4 + (k & 3);
        p[0] = R(0.0);
        p[sstride] = R(0.0);
        p[2 * sstride] = R(0.0);
        p[3 * sstride] = R(0.0);
      }
    }
  };
  if (own >= 0) {
    orderings(std::integral_constant<int, 1>{}, own & 31, own >> 5, out);
  } else {
    // pass states s0 .. s0 + ns - 1: gluon state (s0 + q) / 2, antitop helicity q % 2
#pragma unroll 1
    for (int q = 0; q < ns; q += 2) orderings(std::integral_constant<int, 2>{}, (s0 + q) >> 1, 0, out + (int64_t)(q * 4) * sstride);
  }
}

template <class R> struct G3Mfma;
template <> struct G3Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 step(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct G3Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 step(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// Colour index that lane group g (= lane / 16) supplies at step (s, r) of a
// 16 x 16 x 4 product, chosen so that the four indices a lane supplies for
// block s = rb are the four rows of Z it receives: the FP32 product returns
// rows 4 g + i to lane group g, the FP64 product rows g + 4 i (i = 0..3).
template <class R> __device__ __forceinline__ constexpr int g3_kidx(int s, int g, int r) {
  return std::is_same<R, float>::value ? 16 * s + 4 * g + r : 16 * s + g + 4 * r;
}

// Colour sum of one pass over the nsl slices (a multiple of 4) of the buffer for the nc
// events of the chunk.  C in LDS in A-operand order (exact integer numerators,
// held as FP32): entry ((rb * 8 + s) * 64 + l) * 4 + r holds
// C[16 rb + l % 16][g3_kidx(s, l / 16, r)] (zero beyond the 120 orderings).
// For the MFMA step (s, r) lane l supplies that entry and
// B[g3_kidx(s, l / 16, r)][event l % 16], so the four lane groups cover colour
// indices 16 s .. 16 s + 15 over the four r; the result lane l holds
// Z[g3_kidx(rb, l / 16, i)][event l % 16] in element i, whose matching
// amplitudes are the B values the lane loaded for s = rb.
// first: the pass overwrites me[]; last: it also writes the event weights.
template <class R>
__global__ void __launch_bounds__(CBLOCK) k_g3_colour(const R* __restrict__ amp, int64_t ld, int64_t nc,
                                                      int nsl, int first, int last, double* __restrict__ me,
                                                      const int* __restrict__ idx, const double* __restrict__ wpre,
                                                      double* __restrict__ w, double inv_den) {
  typedef typename G3Mfma<R>::v4 v4;
  typedef float f4 __attribute__((ext_vector_type(4)));
  // 16-event column blocks per tile: two in FP32, one in FP64 (register budget)
  constexpr int NCB = std::is_same<R, float>::value ? 2 : 1;
  constexpr int CTR = 16 * NCB;
  __shared__ float cs[8 * 8 * 64 * 4];
  __shared__ double part[CBLOCK / 64][CT];
  for (int i = threadIdx.x; i < 8 * 8 * 64 * 4; i += CBLOCK) {
    const int r = i & 3, l = (i >> 2) & 63, s = (i >> 8) & 7, rb = i >> 11;
    const int row = 16 * rb + (l & 15), col = g3_kidx<R>(s, l >> 4, r);
    cs[i] = (row < NF && col < NF) ? AMP_M5_COLOUR[row * NF + col] : 0.0f;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, c16 = lane & 15;
  const int64_t ntile = (nc + CTR - 1) / CTR;
  for (int64_t tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    const int64_t c0 = tile * CTR;
    double sum[2] = {0.0, 0.0};
#pragma unroll 1
    for (int sl = wave * (nsl / 4); sl < (wave + 1) * (nsl / 4); ++sl) {
      const R* base = amp + (int64_t)sl * NQ * ld * 4;
      v4 bv[8][NCB];
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          const int64_t col = c0 + 16 * cb + c16;
          if constexpr (std::is_same<R, float>::value) {
            bv[s][cb] = *reinterpret_cast<const v4*>(base + ((int64_t)(4 * s + g) * ld + col) * 4);
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) bv[s][cb][r] = base[((int64_t)(4 * s + r) * ld + col) * 4 + g];
          }
        }
      R acc[2] = {R(0.0), R(0.0)};
#pragma unroll
      for (int rb = 0; rb < 8; ++rb) {
        v4 zz[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) zz[cb] = v4{R(0.0), R(0.0), R(0.0), R(0.0)};
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const f4 a = *reinterpret_cast<const f4*>(&cs[((rb * 8 + s) * 64 + lane) * 4]);
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) zz[cb] = G3Mfma<R>::step(R(a[r]), bv[s][cb][r], zz[cb]);
        }
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[cb] = fma(zz[cb][i], bv[rb][cb][i], acc[cb]);
      }
      sum[0] += (double)acc[0];
      sum[1] += (double)acc[1];
    }
    // the four lane groups hold disjoint rows of the same events
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      sum[cb] += __shfl_xor(sum[cb], 16);
      sum[cb] += __shfl_xor(sum[cb], 32);
    }
    if (g == 0) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) part[wave][16 * cb + c16] = sum[cb];
    }
    __syncthreads();
    if (threadIdx.x < CTR) {
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

#define G3_TRY(expr)                  \
  do {                                \
    hipError_t e_ = (expr);           \
    if (e_ != hipSuccess) return e_;  \
  } while (0)

template <class R>
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
  int64_t want = count < NCMAX_R<R> ? (int64_t)count : NCMAX_R<R>;
  want = (want + AWAVE - 1) / AWAVE * AWAVE;
  if (ws->ld < want) {
    (void)hipFree(ws->d_amp);
    (void)hipFree(ws->d_me);
    ws->d_amp = nullptr;
    ws->d_me = nullptr;
    ws->ld = 0;
    const size_t bytes = sizeof(R) * (size_t)SLICES * NQ * (size_t)want * 4;
    G3_TRY(hipMalloc(&ws->d_amp, bytes));
    G3_TRY(hipMalloc(&ws->d_me, sizeof(double) * want));
    ws->ld = want;
    ws->amp_bytes = bytes;
  }
  const int64_t ld = ws->ld;
  R* amp = static_cast<R*>(ws->d_amp);
  // all states in passes of SP, or one state per point in a single pass
  const bool own = c.helicity != 0;
  const int NPASS = own ? 1 : STATES / SP, ns = own ? 1 : SP, nsl = 4 * ns;
  const double inv_den = (c.helicity == 1 ? (double)STATES : 1.0) / AMP_M5_COLOUR_DEN;
  for (int64_t c0 = 0; c0 < count; c0 += ld) {
    const int64_t nc = (count - c0) < ld ? (count - c0) : ld;
    const int* idx = ws->d_idx + c0;
    const unsigned ablk = (unsigned)((nc + AWAVE - 1) / AWAVE);
    const int64_t ntile = (nc + (std::is_same<R, float>::value ? CT : CT / 2) - 1) /
                          (std::is_same<R, float>::value ? CT : CT / 2);
    const unsigned cblk = (unsigned)(ntile < CMAX_BLOCKS ? ntile : CMAX_BLOCKS);
    for (int pass = 0; pass < NPASS; ++pass) {
      hipLaunchKernelGGL((k_g3_amp<R>), dim3(ablk), dim3(AWAVE), 0, s, c, u, n, idx, nc, pass * SP, ns, amp, ld);
      hipLaunchKernelGGL((k_g3_colour<R>), dim3(cblk), dim3(CBLOCK), 0, s, amp, ld, nc, nsl, pass == 0 ? 1 : 0,
                         pass == NPASS - 1 ? 1 : 0, ws->d_me, idx, ws->d_wpre, w, inv_den);
    }
    G3_TRY(hipGetLastError());
  }
  return hipSuccess;
}

#undef G3_TRY

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

}  // namespace g3
}  // namespace mf
