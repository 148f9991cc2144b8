// Coupling normalising flow (piecewise-quadratic coupling layers, Mueller et
// al. 2019) on gfx950: forward/inverse layer kernel, backward kernels, Adam,
// and the flow part of the C ABI.
//
// Kernels:
//   k_coupling      one coupling layer for a tile of 64 events: the three
//                   dense layers as BF16 MFMA products (v_mfma_f32_16x16x32_bf16,
//                   FP32 accumulation) with the hidden activations resident in
//                   LDS, then the FP32 piecewise-quadratic CDF (or its inverse)
//                   of each transformed coordinate; optionally writes the
//                   activations needed by the backward pass
//   k_pq_backward   derivatives of the PQ transform with respect to its input
//                   and its 2K+1 logits (per event and transformed coordinate)
//   k_gemm          LDS-staged BF16 MFMA product with split-K for the weight
//                   gradients and a LeakyReLU-derivative epilogue for the
//                   activation gradients
//   k_reduce_grad   ordered reduction of the split-K partials into the FP32
//                   gradient
//   k_adam          Adam on the FP32 masters and refresh of the BF16 copies
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/mf_flow.h"
#include "flow_internal.h"
#include "pipeline.h"
#include "status.h"

namespace mf {
namespace flow {

constexpr int H = 256;        // hidden width
constexpr int KB = 32;        // PQ bins
constexpr int NO = 2 * KB + 1;  // logits per transformed coordinate
constexpr int NOP = 80;       // NO padded to five 16-column MFMA tiles
constexpr int KA = 32;        // first-layer k width: inputs split as BF16 hi (k < 16) + lo (k >= 16)
constexpr int KLO = 16;       // offset of the low parts
constexpr int T = 64;         // events per workgroup of the layer kernel
constexpr int LDO = 68;       // LDS row stride (floats) of one coordinate's 64 leading logits (16-byte rows)
constexpr int FMAXD = 16;
constexpr int TBMAX = FMAXD / 2;  // transformed coordinates per layer (the masks take one half)
constexpr int MAXL = 8;
constexpr float SLOPE = 0.01f;

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct LayerDev {
  int dA, dB;
  int a_idx[FMAXD];
  int b_idx[FMAXD];
  const bf16* W1t;   // [H][KA]      (W1 transposed, at k = i and k = KLO + i)
  const float* b1;   // [H]
  const float* b2;   // [H]
  const float* b3p;  // [dB*NOP]
  // The coupling kernel's A fragments of the second layer and of the 64
  // leading logits of the third, packed so that one wave's fragment load is
  // 1 KB of consecutive bytes (64 lanes x 16 B) instead of 16 rows x 64 B;
  // element (k, j) is W[k][j] (input k, output j; the outputs of W3 padded
  // to NOP per coordinate):
  //   W2p[((w * 8 + ks) * 4 + jt) * 64 + lane][8]:  output j = 64 w + 16 jt + (lane & 15),
  //                                                 k = 32 ks + 8 (lane >> 4) + e
  //   W3p[((c * 4 + w) * 8 + ks) * 64 + lane][8]:  output c NOP + 16 w + (lane & 15), same k
  //   W3L[ks * 64 + lane][8]:                    output (lane & 15) NOP + 2K (the 65th
  //                                                 logit of coordinate lane & 15; zero
  //                                                 past d_B), same k
  const bf16* W2p;   // [H][H]
  const bf16* W3p;   // [dB][64][H]
  const bf16* W3L;   // [16][H]
  // The backward products' B operands with k contiguous: W2 [in][out] and
  // W3 [in][dB*NOP] in their own orientation (zero-padded outputs)
  const bf16* W2n;   // [H][H]
  const bf16* W3n;   // [H][dB*NOP]
};

// Training caches of one layer.  The activations are kept event-contiguous
// ([feature][ldn], ldn = the batch rounded up to 8) because their only
// consumers are the weight-gradient products, which reduce over events.
struct LayerCache {
  bf16* xa;     // [KA][ldn] inputs of the first dense layer (hi | lo)
  bf16* h1;     // [H][ldn]
  bf16* h2;     // [H][ldn]
  float* o;     // [n][dB][NOP] logits
  float* lin;   // [d][n]   layer input
  int64_t ldn;  // leading dimension of the event-contiguous caches
};

__device__ __forceinline__ f32x4 mfma16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Hidden activations in LDS: [T][H] bf16 with the 16-byte chunks of a row
// permuted by the row index, so that the 16 rows read by one fragment load
// fall in different banks.
__device__ __forceinline__ int hs(int m, int k) { return m * H + ((((k >> 3) ^ (m & 15))) << 3) + (k & 7); }

// The median of (v, 0.01 v, FLT_MAX) is max(v, 0.01 v) for finite v: v for v >= 0 and 0.01 v
// below, the LeakyReLU in two operations (fmaxf would add a canonicalising
// instruction per input in IEEE mode)
__device__ __forceinline__ float leaky(float v) { return __builtin_amdgcn_fmed3f(v, SLOPE * v, 3.40282347e38f); }

// Exchanges inside an aligned group of four lanes through DPP quad
// permutations (no LDS round trip): lane ^ 1, lane ^ 2, and the group's lane
// 0, 1 or 2 broadcast to all four.  A quad permutation reads a lane of the
// same group for every lane, so no old value is needed.
constexpr int QX1 = 0xB1, QX2 = 0x4E, QB0 = 0x00, QB1 = 0x55, QB2 = 0xAA;
template <int CTRL> __device__ __forceinline__ float qdpp(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, true));
}
template <int CTRL> __device__ __forceinline__ int qdpp(int x) {
  return __builtin_amdgcn_mov_dpp(x, CTRL, 0xF, 0xF, true);
}
// max(a, b) of finite values as the median of (a, b, FLT_MAX), without the
// canonicalising instructions fmaxf adds in IEEE mode
__device__ __forceinline__ float max_nc(float a, float b) {
  return __builtin_amdgcn_fmed3f(a, b, 3.40282347e38f);
}

// ------------------------------------------------------------ PQ transform
// Softmax widths and normalised vertex heights from the 2K+1 logits.
__device__ __forceinline__ void pq_params(const float* o, float* W, float* V) {
  float mw = o[0];
#pragma unroll
  for (int k = 1; k < KB; ++k) mw = fmaxf(mw, o[k]);
  float sw = 0.0f;
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    W[k] = __expf(o[k] - mw);
    sw += W[k];
  }
  const float isw = 1.0f / sw;
#pragma unroll
  for (int k = 0; k < KB; ++k) W[k] *= isw;
  float mv = o[KB];
#pragma unroll
  for (int k = 1; k <= KB; ++k) mv = fmaxf(mv, o[KB + k]);
#pragma unroll
  for (int k = 0; k <= KB; ++k) V[k] = __expf(o[KB + k] - mv);
  float N = 0.0f;
#pragma unroll
  for (int k = 0; k < KB; ++k) N += 0.5f * (V[k] + V[k + 1]) * W[k];
  const float iN = 1.0f / N;
#pragma unroll
  for (int k = 0; k <= KB; ++k) V[k] *= iN;
}

// Bin b of a point: the largest k >= 1 with edge_k <= t (else 0), where
// edge_k is the running sum of W (by_area = 0) or of the bin areas
// (by_area = 1).  Returns the bin's left edge S_b, its area offset A_b,
// W_b, V_b, V_b+1 through static register indices only.
struct Bin {
  int b;
  float S, A, Wb, Vb, Vb1;
};
__device__ __forceinline__ Bin find_bin(const float* W, const float* V, float t, bool by_area) {
  Bin r{0, 0.0f, 0.0f, W[0], V[0], V[1]};
  float S = W[0], A = 0.5f * (V[0] + V[1]) * W[0];
#pragma unroll
  for (int k = 1; k < KB; ++k) {
    const bool take = (by_area ? A : S) <= t;
    r.b = take ? k : r.b;
    r.S = take ? S : r.S;
    r.A = take ? A : r.A;
    r.Wb = take ? W[k] : r.Wb;
    r.Vb = take ? V[k] : r.Vb;
    r.Vb1 = take ? V[k + 1] : r.Vb1;
    S += W[k];
    A += 0.5f * (V[k] + V[k + 1]) * W[k];
  }
  return r;
}

// Epilogue of a transposed dense layer: acc[jt][mt][i] is feature
// 64 wave + 16 jt + 4 quad + i of event 16 mt + row, bias included (it is
// the accumulator's initial value); applies the LeakyReLU, rounds to BF16 and
// stores the four features with one 8-byte write into the permuted [T][H]
// activation tile.
__device__ __forceinline__ void store_features(bf16* h, const f32x4 (&acc)[4][4], int wave, int row, int quad) {
#pragma unroll
  for (int jt = 0; jt < 4; ++jt) {
    const int f0 = 64 * wave + 16 * jt + 4 * quad;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      bf16x4 v;
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = (bf16)leaky(acc[jt][mt][i]);
      *reinterpret_cast<bf16x4*>(h + hs(16 * mt + row, f0)) = v;
    }
  }
}

// The bias of the four features 64 wave + 16 jt + 4 quad + i (i = 0..3) as an
// accumulator tile.
__device__ __forceinline__ f32x4 bias4(const float* __restrict__ b, int wave, int jt, int quad) {
  const float* p = b + 64 * wave + 16 * jt + 4 * quad;
  return f32x4{p[0], p[1], p[2], p[3]};
}

// The PQ transform of one coordinate with four lanes per event: lane part p
// holds the bins [8p, 8p+8) and the vertices [8p, 8p+8] of the 2K+1 logits
// (the first 2K in LDS at o, the last one, vlast, in a register of the
// p = 3 lane); maxima, sums, prefix offsets and the bin's owner are combined
// with DPP quad exchanges.  Same bin rule as find_bin: the largest k >= 1
// whose left edge (running width, or running area for the sampling
// direction) is <= t, else 0.  Every lane of the group returns the result
// (y or z) and the density.  Reciprocals use the hardware approximation
// (1 ulp).
template <bool INVERSE>
__device__ __forceinline__ void pq_quad(const float* o, float vlast, float t, int p, float& res, float& pdf) {
  constexpr int KP = KB / 4;
  float w[KP], v[KP + 1];
#pragma unroll
  for (int k = 0; k < KP; ++k) w[k] = o[KP * p + k];
#pragma unroll
  for (int k = 0; k < KP; ++k) v[k] = o[KB + KP * p + k];
  {
    // the part's last vertex: the next part's first, or the 2K+1-th logit
    const float vn = o[KB + KP * p + (p < 3 ? KP : 0)];
    v[KP] = p < 3 ? vn : vlast;
  }
  // exp(x - m) as 2^(x log2 e - m log2 e), one FMA and the hardware exp2
  constexpr float L2E = 1.4426950408889634f;
  float mw = w[0];
#pragma unroll
  for (int k = 1; k < KP; ++k) mw = fmaxf(mw, w[k]);
  mw = max_nc(mw, qdpp<QX1>(mw));
  mw = max_nc(mw, qdpp<QX2>(mw));
  const float mwl = mw * L2E;
  // the widths stay unnormalised (sum sw); the part's sum is its offset
  float sw = 0.0f;
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    w[k] = __builtin_amdgcn_exp2f(fmaf(w[k], L2E, -mwl));
    sw += w[k];
  }
  const float part_w = sw;
  sw += qdpp<QX1>(sw);
  sw += qdpp<QX2>(sw);
  float mv = v[0];
#pragma unroll
  for (int k = 1; k <= KP; ++k) mv = fmaxf(mv, v[k]);
  mv = max_nc(mv, qdpp<QX1>(mv));
  mv = max_nc(mv, qdpp<QX2>(mv));
  const float mvl = mv * L2E;
#pragma unroll
  for (int k = 0; k <= KP; ++k) v[k] = __builtin_amdgcn_exp2f(fmaf(v[k], L2E, -mvl));
  // bin areas with the unnormalised widths and heights, twice over:
  // ar_k = (v_k + v_k+1) w_k, total nl
  float ar[KP];
  float nl = 0.0f;
#pragma unroll
  for (int k = 0; k < KP; ++k) {
    ar[k] = (v[k] + v[k + 1]) * w[k];
    nl += ar[k];
  }
  const float part_a = nl;
  nl += qdpp<QX1>(nl);
  nl += qdpp<QX2>(nl);
  // normalised: width w_k / sw, area ar_k / nl, height v_k 2 sw / nl (unit
  // total area); the running edges are compared in unnormalised units
  const float isw = __builtin_amdgcn_rcpf(sw);
  const float iar = __builtin_amdgcn_rcpf(nl);
  const float tt = t * (INVERSE ? nl : sw);
  // exclusive offsets of the running width and area at the part's first bin
  const float s0 = qdpp<QB0>(part_w), s1 = qdpp<QB1>(part_w), s2 = qdpp<QB2>(part_w);
  const float a0 = qdpp<QB0>(part_a), a1 = qdpp<QB1>(part_a), a2 = qdpp<QB2>(part_a);
  float S = (p > 0 ? s0 : 0.0f) + (p > 1 ? s1 : 0.0f) + (p > 2 ? s2 : 0.0f);
  float A = (p > 0 ? a0 : 0.0f) + (p > 1 ? a1 : 0.0f) + (p > 2 ? a2 : 0.0f);
  // the edges grow with the bin index, so bin b is owned by the last lane
  // of the group whose first bin is taken
  const bool first = p == 0 || (INVERSE ? A : S) <= tt;
  int owner = first ? p : -1;
  float Sb = S, Ab = A, Wb = w[0], Vb = v[0], Vb1 = v[1];
  S += w[0];
  A += ar[0];
#pragma unroll
  for (int k = 1; k < KP; ++k) {
    const bool take = (INVERSE ? A : S) <= tt;
    Sb = take ? S : Sb;
    Ab = take ? A : Ab;
    Wb = take ? w[k] : Wb;
    Vb = take ? v[k] : Vb;
    Vb1 = take ? v[k + 1] : Vb1;
    S += w[k];
    A += ar[k];
  }
  owner = max(owner, qdpp<QX1>(owner));
  owner = max(owner, qdpp<QX2>(owner));
  Sb *= isw;
  Ab *= iar;
  Wb *= isw;
  const float hn = 2.0f * sw * iar;
  Vb *= hn;
  Vb1 *= hn;
  const float dV = Vb1 - Vb;
  const float iW = __builtin_amdgcn_rcpf(Wb);
  float r, q;
  if (!INVERSE) {
    const float al = fminf(fmaxf((t - Sb) * iW, 0.0f), 1.0f);
    r = Ab + Wb * (al * Vb + 0.5f * al * al * dV);
    q = Vb + al * dV;
  } else {
    const float cc = (t - Ab) * iW;
    const float disc = fmaxf(Vb * Vb + 2.0f * dV * cc, 0.0f);
    // hardware square root (1 ulp)
    float al = 2.0f * cc * __builtin_amdgcn_rcpf(Vb + __builtin_amdgcn_sqrtf(disc));
    al = fminf(fmaxf(al, 0.0f), 1.0f);
    r = Sb + al * Wb;
    q = Vb + al * dV;
  }
  // only the owner of bin b holds the right values: a sum over the group
  // with the other three lanes contributing exact zeros
  const bool own = owner == p;
  float rr = own ? r : 0.0f, qq = own ? q : 0.0f;
  rr += qdpp<QX1>(rr);
  qq += qdpp<QX1>(qq);
  res = rr + qdpp<QX2>(rr);
  pdf = qq + qdpp<QX2>(qq);
}

// --------------------------------------------------------- coupling layer
// Copy of the [T][H] activation tile into an event-contiguous cache: eight
// events of one feature per 16-byte store.
__device__ __forceinline__ void cache_hidden(const bf16* h, bf16* __restrict__ dst, int64_t ldn, int64_t e0,
                                             int64_t n, int tid) {
  for (int idx = tid; idx < H * (T / 8); idx += 256) {
    const int ch = idx % (T / 8), f = idx / (T / 8);
    const int m0 = 8 * ch;
    const int64_t e = e0 + m0;
    if (e >= n) continue;
    bf16x8 v;
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = h[hs(m0 + i, f)];
    if (e + 8 <= n) {
      *reinterpret_cast<bf16x8*>(dst + (int64_t)f * ldn + e) = v;
    } else {
      for (int i = 0; e + i < n; ++i) dst[(int64_t)f * ldn + e + i] = v[i];
    }
  }
}

// One layer for events [64 blockIdx.x, +64): y is [d][ld] (n <= ld events
// used) and is transformed in place (the kept coordinates are only read).
// INVERSE selects the sampling direction.  logq[e] is set (first layer) or
// accumulated.  The caches use row length n.
//
// LDS: one [T][H] BF16 tile that holds the first hidden layer and then the
// second (written over the first once every wave has read it), and one
// [T][LDO] FP32 tile for the 64 leading logits of the current coordinate
// (before that, its first 4 KB hold the first-layer inputs), and the inputs
// of the transformed coordinates (2 KiB): 51.0 KiB, so that three
// workgroups share a compute unit.
template <bool INVERSE, bool CACHE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CACHE ? 2 : 3))) k_coupling(LayerDev L, float* __restrict__ y, int64_t n, int64_t ld,
                                                  float* __restrict__ logq, int first, LayerCache C, int d) {
  __shared__ __attribute__((aligned(16))) bf16 h[T * H];
  __shared__ __attribute__((aligned(16))) float out[T * LDO];
  __shared__ float tb[TBMAX * T];
  static_assert(T * KA * sizeof(bf16) <= T * LDO * sizeof(float), "first-layer inputs must fit the logit tile");
  bf16* xa = reinterpret_cast<bf16*>(out);  // [T][KA]
  // the wave index is uniform across the wave: held in a scalar register, the
  // per-wave weight and index addresses are scalar arithmetic
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t e0 = (int64_t)blockIdx.x * T;
  const int row = lane & 15, quad = lane >> 4;

  // inputs of the first dense layer (events fastest, so the reads coalesce):
  // each kept coordinate as a BF16 pair hi + lo (about 16 significant bits),
  // multiplied by the same weight column
  {
    // all of this thread's HBM reads are issued before the first is used
    // (one latency instead of several): kept coordinates w, w + 4, w + 8,
    // w + 12 and transformed coordinates w, w + 4 of event m (w = wave); the
    // transformed ones wait in LDS for their PQ transforms
    static_assert(KLO == 16 && TBMAX == 8, "four kept and two transformed coordinates per thread");
    const int m = lane;
    const int64_t e = e0 + m;
    const bool ev = e < n;
    float v[4], tv[2];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = wave + 4 * r;
      v[r] = (i < L.dA && ev) ? y[(int64_t)L.a_idx[i] * ld + e] : 0.0f;
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int j = wave + 4 * r;
      tv[r] = (j < L.dB && ev) ? y[(int64_t)L.b_idx[j] * ld + e] : 0.5f;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = wave + 4 * r;
      const bf16 hi = (bf16)v[r];
      const bf16 lo = (bf16)(v[r] - (float)hi);
      const int il = i + KLO;
      xa[m * KA + (((i >> 3) ^ (m & 3)) << 3) + (i & 7)] = hi;
      xa[m * KA + (((il >> 3) ^ (m & 3)) << 3) + (il & 7)] = lo;
      if (CACHE && ev) {
        C.xa[i * C.ldn + e] = hi;
        C.xa[il * C.ldn + e] = lo;
      }
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int j = wave + 4 * r;
      if (j < L.dB) tb[j * T + m] = tv[r];
    }
  }
  if (CACHE) {
    for (int idx = tid; idx < T * d; idx += 256) {
      const int m = idx % T, j = idx / T;
      const int64_t e = e0 + m;
      if (e < n) C.lin[(int64_t)j * n + e] = y[(int64_t)j * ld + e];
    }
  }
  __syncthreads();

  // Dense layers 1 and 2 are computed transposed, D[feature][event] =
  // W^T X^T: the weight rows are the A fragments (16-byte loads from the
  // [out][in] copies), the activations in LDS the B fragments, and each lane
  // ends with four consecutive features of one event, stored as one 8-byte
  // LDS write after bias and activation.  Wave w owns features [64w, 64w+64).
  {
    f32x4 acc[4][4];
    bf16x8 a[4], b[4];
#pragma unroll
    for (int jt = 0; jt < 4; ++jt)
      a[jt] = *reinterpret_cast<const bf16x8*>(L.W1t + (64 * wave + 16 * jt + row) * KA + 8 * quad);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      const int m = 16 * mt + row;
      b[mt] = *reinterpret_cast<const bf16x8*>(xa + m * KA + ((quad ^ (m & 3)) << 3));
    }
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) {
      const f32x4 bias = bias4(L.b1, wave, jt, quad);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) acc[jt][mt] = mfma16(a[jt], b[mt], bias);
    }
    store_features(h, acc, wave, row, quad);
  }
  __syncthreads();
  if (CACHE) cache_hidden(h, C.h1, C.ldn, e0, n, tid);
  {
    f32x4 acc[4][4];
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) {
      const f32x4 bias = bias4(L.b2, wave, jt, quad);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) acc[jt][mt] = bias;
    }
    // this wave's fragments in packed order: step ks, fragment jt at
    // ((wave 8 + ks) 4 + jt) KB; a step's fragments are requested two steps
    // ahead (a ring of three) and kept in their step by a scheduling barrier
    const bf16* W2 = L.W2p + (int64_t)wave * 8 * 4 * 512 + lane * 8;
    bf16x8 a[3][4];
#pragma unroll
    for (int st = 0; st < 2; ++st)
#pragma unroll
      for (int jt = 0; jt < 4; ++jt) a[st][jt] = *reinterpret_cast<const bf16x8*>(W2 + (st * 4 + jt) * 512);
#pragma unroll
    for (int ks = 0; ks < H / 32; ++ks) {
      if (ks + 2 < H / 32) {
#pragma unroll
        for (int jt = 0; jt < 4; ++jt)
          a[(ks + 2) % 3][jt] = *reinterpret_cast<const bf16x8*>(W2 + ((ks + 2) * 4 + jt) * 512);
      }
      bf16x8 b[4];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
        b[mt] = *reinterpret_cast<const bf16x8*>(h + hs(16 * mt + row, 32 * ks + 8 * quad));
#pragma unroll
      for (int jt = 0; jt < 4; ++jt)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc[jt][mt] = mfma16(a[ks % 3][jt], b[mt], acc[jt][mt]);
      __builtin_amdgcn_sched_barrier(0);
    }
    // every wave has read the first layer (and the cache copy is done)
    // before the second overwrites it
    __syncthreads();
    store_features(h, acc, wave, row, quad);
  }
  __syncthreads();
  if (CACHE) cache_hidden(h, C.h2, C.ldn, e0, n, tid);

  // The 65th logit of every transformed coordinate at once: one more MFMA
  // tile per wave, D[coordinate][event] for the wave's 16 events, with the
  // weight rows of the coordinates' last outputs as A fragments (packed;
  // rows past d_B are zero and never read).  Lane l keeps coordinates
  // 4 (l >> 4) + i of event 16 wave + (l & 15) in registers until their PQ
  // transforms.
  f32x4 lastv = {0.0f, 0.0f, 0.0f, 0.0f};
  {
    const bf16* wl = L.W3L + lane * 8;
#pragma unroll
    for (int ks = 0; ks < H / 32; ++ks) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(wl + ks * 512);
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(h + hs(16 * wave + row, 32 * ks + 8 * quad));
      lastv = mfma16(a, b, lastv);
    }
  }

  // dense layer 3 and the PQ transform, one transformed coordinate at a time:
  // the 64 leading logits of a coordinate are four 16-column MFMA tiles, one
  // per wave over all 64 events (each wave streams only its own weight
  // columns).
  float lq = 0.0f;
  // the eight weight fragments of this wave's columns of coordinate c; those
  // of coordinate c + 1 are requested before the PQ transform of c, so their
  // L2 latency overlaps it
  bf16x8 bw[H / 32];
  {
    const bf16* W3 = L.W3p + (int64_t)wave * 8 * 512 + lane * 8;
#pragma unroll
    for (int ks = 0; ks < H / 32; ++ks) bw[ks] = *reinterpret_cast<const bf16x8*>(W3 + ks * 512);
  }
  // the PQ transform's event (16 per wave, four lanes each) and part
  const int m = tid >> 2, part = tid & 3;
  const int64_t em = e0 + m;
  const bool live = em < n;
  for (int c = 0; c < L.dB; ++c) {
    {
      const int col = 16 * wave + row;
      const float bias = L.b3p[c * NOP + col];
      f32x4 acc[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = f32x4{bias, bias, bias, bias};
#pragma unroll
      for (int ks = 0; ks < H / 32; ++ks) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const bf16x8 a = *reinterpret_cast<const bf16x8*>(h + hs(16 * r + row, 32 * ks + 8 * quad));
          acc[r] = mfma16(a, bw[ks], acc[r]);
        }
      }
      if (c + 1 < L.dB) {
        const bf16* W3 = L.W3p + (((int64_t)(c + 1) * 4 + wave) * 8) * 512 + lane * 8;
#pragma unroll
        for (int ks = 0; ks < H / 32; ++ks) bw[ks] = *reinterpret_cast<const bf16x8*>(W3 + ks * 512);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) out[(16 * r + 4 * quad + i) * LDO + col] = acc[r][i];
    }
    // the 65th logit of (event m, coordinate c) from the lane of this wave
    // that holds it
    const int ci = c & 3;
    const float lsel = ci == 0 ? lastv[0] : ci == 1 ? lastv[1] : ci == 2 ? lastv[2] : lastv[3];
    const float vlast = __shfl(lsel, (lane >> 2) + 16 * (c >> 2)) + L.b3p[c * NOP + 2 * KB];
    __syncthreads();
    if (CACHE) {
      for (int idx = tid; idx < T * 2 * KB; idx += 256) {
        const int mm = idx / (2 * KB), col = idx % (2 * KB);
        const int64_t e = e0 + mm;
        if (e < n) C.o[(e * L.dB + c) * NOP + col] = out[mm * LDO + col];
      }
      if (live && part == 3) C.o[(em * L.dB + c) * NOP + 2 * KB] = vlast;
    }
    {
      float* yp = y + (int64_t)L.b_idx[c] * ld + (live ? em : e0);
      const float t = tb[c * T + m];
      float res, pdf;
      pq_quad<INVERSE>(out + m * LDO, vlast, t, part, res, pdf);
      if (live && part == 0) {
        *yp = res;
        lq += __logf(pdf);
      }
    }
    __syncthreads();
  }
  if ((tid & 3) == 0) {
    const int64_t e = e0 + (tid >> 2);
    if (e < n) logq[e] = first ? lq : logq[e] + lq;
  }
}

// ------------------------------------------------------------ PQ backward
// For event e = 256 blockIdx.x + threadIdx.x and transformed coordinate
// c = blockIdx.y: given the gradient gz of the loss with respect to the layer
// output at that coordinate (g[j][e]) and glp = dL/dlog q = -w_e / sum w,
// replaces g[j][e] by the gradient with respect to the layer input and writes
// the gradient with respect to the 2K+1 logits (BF16, padded to NOP with
// zeros), row-major per event and event-contiguous per logit (through an LDS
// tile, 16-byte stores).
__global__ void __launch_bounds__(256) k_pq_backward(LayerDev L, LayerCache C, int64_t n, float* __restrict__ g,
                                                     const float* __restrict__ w, const float* __restrict__ wsum,
                                                     bf16* __restrict__ go, bf16* __restrict__ goT) {
  __shared__ __attribute__((aligned(16))) bf16 tile[NOP][256 + 8];
  const int c = blockIdx.y;
  const int64_t eb = (int64_t)blockIdx.x * 256;
  const int64_t e = eb + threadIdx.x;
  const bool live = e < n;
  if (live) {
  const int j = L.b_idx[c];
  const float* o = C.o + (e * L.dB + c) * NOP;
  float ol[NO];
#pragma unroll
  for (int k = 0; k < NO; ++k) ol[k] = o[k];
  float W[KB], V[KB + 1];
  pq_params(ol, W, V);
  const float yv = C.lin[(int64_t)j * n + e];
  const Bin B = find_bin(W, V, yv, false);
  const float al = fminf(fmaxf((yv - B.S) / B.Wb, 0.0f), 1.0f);
  const float dV = B.Vb1 - B.Vb;
  const float pdf = B.Vb + al * dV;
  const float gz = g[(int64_t)j * n + e];
  const float glp = -w[e] / wsum[0];
  const float gp = glp / pdf;
  // d/dW_k and d/dV_k of (gz z + glp log pdf) at fixed logits of other bins
  float GW[KB], GV[KB + 1];
#pragma unroll
  for (int k = 0; k <= KB; ++k) GV[k] = 0.0f;
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const bool below = k < B.b, at = k == B.b;
    const float dz = below ? 0.5f * (V[k] + V[k + 1]) - B.Vb - al * dV : (at ? -0.5f * al * al * dV : 0.0f);
    const float dp = below ? -dV / B.Wb : (at ? -al * dV / B.Wb : 0.0f);
    GW[k] = gz * dz + gp * dp;
    // area terms of z: A_b = sum_{k<b} W_k (V_k + V_k+1)/2
    if (below) {
      GV[k] += gz * 0.5f * W[k];
      GV[k + 1] += gz * 0.5f * W[k];
    }
  }
#pragma unroll
  for (int k = 0; k <= KB; ++k) {
    const bool at = k == B.b, next = k == B.b + 1;
    GV[k] += at ? gz * B.Wb * (al - 0.5f * al * al) + gp * (1.0f - al) : 0.0f;
    GV[k] += next ? gz * B.Wb * 0.5f * al * al + gp * al : 0.0f;
  }
  g[(int64_t)j * n + e] = gz * pdf + glp * (dV / B.Wb) / pdf;
  // through V = exp(v) / N, N = sum_k W_k (exp(v_k) + exp(v_k+1)) / 2, and W = softmax
  float SG = 0.0f;
#pragma unroll
  for (int k = 0; k <= KB; ++k) SG += GV[k] * V[k];
  float SW = 0.0f;
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    GW[k] -= SG * 0.5f * (V[k] + V[k + 1]);
    SW += W[k] * GW[k];
  }
  // row-major for the activation-gradient product, event-contiguous for the
  // weight-gradient product
  bf16* dst = go + e * ((int64_t)L.dB * NOP) + (int64_t)c * NOP;
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const bf16 v = (bf16)(W[k] * (GW[k] - SW));
    dst[k] = v;
    tile[k][threadIdx.x] = v;
  }
#pragma unroll
  for (int k = 0; k <= KB; ++k) {
    const float wl = k > 0 ? W[k - 1] : 0.0f, wr = k < KB ? W[k] : 0.0f;
    const bf16 v = (bf16)(V[k] * (GV[k] - SG * 0.5f * (wl + wr)));
    dst[KB + k] = v;
    tile[KB + k][threadIdx.x] = v;
  }
#pragma unroll
  for (int k = NO; k < NOP; ++k) {
    dst[k] = (bf16)0.0f;
    tile[k][threadIdx.x] = (bf16)0.0f;
  }
  }
  __syncthreads();
  // event-contiguous copy: 8 events of one logit per 16-byte store
  bf16* dstT = goT + (int64_t)c * NOP * C.ldn;
  for (int ch = threadIdx.x; ch < NOP * 32; ch += 256) {
    const int k = ch / 32, e8 = 8 * (ch % 32);
    const int64_t ee = eb + e8;
    if (ee >= n) continue;
    const bf16x8 v = *reinterpret_cast<const bf16x8*>(&tile[k][e8]);
    if (ee + 8 <= n) {
      *reinterpret_cast<bf16x8*>(dstT + (int64_t)k * C.ldn + ee) = v;
    } else {
      for (int i = 0; ee + i < n; ++i) dstT[(int64_t)k * C.ldn + ee + i] = v[i];
    }
  }
}

// ------------------------------------------------------------------ GEMM
// C[M x N] = sum over k in the z-th chunk of A(m,k) B(k,n), BF16 operands,
// FP32 accumulation, tile 64 x 64 per workgroup, k-step 32 staged in LDS.
//   A_KC: A(m,k) = A[m lda + k] (1) or A[k lda + m] (0)
//   B_NC: B(k,n) = B[k ldb + n] (1) or B[n ldb + k] (0)
//   EPI 0: FP32 store to Cf + z zs + m ldc + n (split-K partials); with
//          colsum set, row M of the partial receives the column sums of B
//          over the chunk (one more MFMA per k-step with an all-ones A
//          fragment in the first row of blocks)
//   EPI 1: BF16 store to Cb[m ldc + n] of acc * (ref[m + n ref_cs] > 0 ? 1 : slope),
//          and of the same values to CbT[n ldt + m] (event-contiguous copy);
//          the references are event-contiguous (ref_rs = 1), and Cb, CbT and
//          ref rows are 16-byte aligned
struct GemmArgs {
  const bf16* A;
  int64_t lda;
  const bf16* B;
  int64_t ldb;
  int M, N;
  int64_t K, kchunk;
  float* Cf;
  int64_t zs;
  bf16* Cb;
  const bf16* ref;
  int64_t ldc, ref_rs, ref_cs;
  bf16* CbT;
  int64_t ldt;
  int colsum;
};

constexpr int GK = 64;        // k depth of one staged slice
constexpr int GLD = GK + 8;   // LDS row stride (bf16) of a staged slice

// C = A B over k in [kchunk z, kchunk (z+1)) for the 64 x 64 output tile of
// the workgroup; four waves of 32 x 32, v_mfma_f32_16x16x32_bf16.  A is
// staged from k-contiguous rows A[m lda + k]; B from B[n ldb + k] (B_NC = 0)
// or B[k ldb + n] (B_NC = 1, transposed into LDS).  The k slices are double
// buffered: the next slice's global loads are issued into registers before
// the current slice's products, and each slice costs one barrier.
template <int A_KC, int B_NC, int EPI>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_gemm(GemmArgs g) {
  static_assert(A_KC == 1, "A is staged from k-contiguous rows");
  // the two double-buffered slices; after the k loop the same memory holds
  // the FP32 output tile of the BF16 epilogue
  __shared__ __attribute__((aligned(16))) bf16 smem[4 * 64 * GLD];
  bf16(*As)[64 * GLD] = reinterpret_cast<bf16(*)[64 * GLD]>(smem);
  bf16(*Bs)[64 * GLD] = reinterpret_cast<bf16(*)[64 * GLD]>(smem + 2 * 64 * GLD);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row = lane & 15, quad = lane >> 4;
  // XCD-aware tile order: workgroup b runs on XCD b mod 8, so the tiles are
  // numbered XCD by XCD; consecutive tiles (the column tiles of one row
  // tile, the tiles of one event chunk) then share an XCD and its L2, and
  // their common operand rows are read from HBM once
  int tx, ty, tz;
  {
    const int gx = gridDim.x, gy = gridDim.y;
    const int G = gx * gy * gridDim.z;
    const int b = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const int xcd = b & 7, slot = b >> 3, per = G >> 3, rem = G & 7;
    const int t = xcd * per + (xcd < rem ? xcd : rem) + slot;
    tx = t % gx;
    ty = (t / gx) % gy;
    tz = t / (gx * gy);
  }
  const int m0 = ty * 64, n0 = tx * 64;
  const int64_t kb = (int64_t)tz * g.kchunk;
  const int64_t ke = kb + g.kchunk < g.K ? kb + g.kchunk : g.K;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  f32x4 accs[2] = {f32x4{0.0f, 0.0f, 0.0f, 0.0f}, f32x4{0.0f, 0.0f, 0.0f, 0.0f}};
  const bool sums = EPI == 0 && g.colsum && ty == 0 && wm == 0;
  bf16x8 ones;
#pragma unroll
  for (int i = 0; i < 8; ++i) ones[i] = (bf16)1.0f;
  // this thread's share of a slice: rows (or k) r0 and r0 + 32, eight
  // consecutive elements from c8, one 16-byte load each.  The loads have no
  // branches (so that the waits for a slice do not wait for the next one):
  // rows and chunks outside the operand read an in-range chunk instead, and
  // the number of valid elements of each chunk (0-8) zeroes the rest when
  // the slice is stored.  The caller guarantees 16-byte aligned rows: base
  // and leading dimension multiples of 8 elements, so a chunk that starts
  // inside a row ends inside it.
  const int r0 = tid >> 3, c8 = (tid & 7) * 8;
  // two register stages: the slices k + 1 and k + 2 are in flight while
  // slice k is multiplied
  bf16x8 ra0[2], rb0[2], ra1[2], rb1[2];
  // valid elements of this thread's A and B chunks h of the slice at k0
  auto nvalid = [](int64_t lim, int64_t j) -> int {
    const int64_t r = lim - j;
    return r <= 0 ? 0 : (r >= 8 ? 8 : (int)r);
  };
  auto va = [&](int64_t k0, int h) -> int { return m0 + r0 + 32 * h < g.M ? nvalid(ke, k0 + c8) : 0; };
  auto vb = [&](int64_t k0, int h) -> int {
    if (B_NC) return k0 + r0 + 32 * h < ke ? nvalid(g.N, n0 + c8) : 0;
    return n0 + r0 + 32 * h < g.N ? nvalid(ke, k0 + c8) : 0;
  };
  auto load = [&](int64_t k0, bf16x8 (&ra)[2], bf16x8 (&rb)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int gm = m0 + r0 + 32 * h;
      ra[h] = *reinterpret_cast<const bf16x8*>(g.A + (int64_t)(gm < g.M ? gm : 0) * g.lda + (va(k0, h) > 0 ? k0 + c8 : kb));
      if (B_NC) {
        const int64_t gk = k0 + r0 + 32 * h;
        rb[h] = *reinterpret_cast<const bf16x8*>(g.B + (gk < ke ? gk : kb) * g.ldb + (vb(k0, h) > 0 ? n0 + c8 : 0));
      } else {
        const int gn = n0 + r0 + 32 * h;
        rb[h] = *reinterpret_cast<const bf16x8*>(g.B + (int64_t)(gn < g.N ? gn : 0) * g.ldb + (vb(k0, h) > 0 ? k0 + c8 : kb));
      }
    }
  };
  // A rows m-major, B rows n-major in LDS, each row GK consecutive k
  auto store = [&](int buf, bf16x8 (&ra)[2], bf16x8 (&rb)[2], int64_t k0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int na = va(k0, h), nb = vb(k0, h);
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        ra[h][i] = i < na ? ra[h][i] : (bf16)0.0f;
        rb[h][i] = i < nb ? rb[h][i] : (bf16)0.0f;
      }
      *reinterpret_cast<bf16x8*>(&As[buf][(r0 + 32 * h) * GLD + c8]) = ra[h];
      if (B_NC) {
#pragma unroll
        for (int i = 0; i < 8; ++i) Bs[buf][(c8 + i) * GLD + r0 + 32 * h] = rb[h][i];
      } else {
        *reinterpret_cast<bf16x8*>(&Bs[buf][(r0 + 32 * h) * GLD + c8]) = rb[h];
      }
    }
  };
  auto products = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < GK; kk += 32) {
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        a[i] = *reinterpret_cast<const bf16x8*>(&As[buf][(wm + 16 * i + row) * GLD + kk + 8 * quad]);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        b[j] = *reinterpret_cast<const bf16x8*>(&Bs[buf][(wn + 16 * j + row) * GLD + kk + 8 * quad]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma16(a[i], b[j], acc[i][j]);
      if (sums) {
#pragma unroll
        for (int j = 0; j < 2; ++j) accs[j] = mfma16(ones, b[j], accs[j]);
      }
    }
  };
  // slices alternate between the register stages and the LDS buffers; the
  // buffer written for a slice was last read two slices before, ahead of the
  // previous slice's barrier.  Each iteration takes two slices and issues the
  // loads of the two after them (empty past the chunk, reading its first
  // columns), so that every iteration has the same loads in flight; an odd
  // last slice follows the loop.
  load(kb, ra0, rb0);
  load(kb + GK, ra1, rb1);
  int64_t k0 = kb;
  for (; k0 + GK < ke; k0 += 2 * GK) {
    store(0, ra0, rb0, k0);
    __syncthreads();
    load(k0 + 2 * GK, ra0, rb0);
    products(0);
    store(1, ra1, rb1, k0 + GK);
    __syncthreads();
    load(k0 + 3 * GK, ra1, rb1);
    products(1);
  }
  if (k0 < ke) {
    store(0, ra0, rb0, k0);
    __syncthreads();
    products(0);
  }
  if (sums && quad == 0) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int gn = n0 + wn + 16 * j + row;
      if (gn < g.N) g.Cf[(int64_t)tz * g.zs + (int64_t)g.M * g.ldc + gn] = accs[j][0];
    }
  }
  if (EPI == 0) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int gn = n0 + wn + 16 * j + row;
        if (gn >= g.N) continue;
        const int gm0 = m0 + wm + 16 * i + 4 * quad;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (gm0 + r < g.M) g.Cf[(int64_t)tz * g.zs + (int64_t)(gm0 + r) * g.ldc + gn] = acc[i][j][r];
      }
  } else {
    // The tile goes through LDS (FP32, row stride LDT: the fragment stores
    // at most two-way bank conflicts, the column reads none), so that the
    // sign references are read and both BF16 copies written with 16-byte
    // accesses: first eight consecutive events of one feature per thread
    // (references, scaling, the event-contiguous copy; the rounded values go
    // back to the tile), then eight consecutive features of one event (the
    // row-major copy).  The references are event-contiguous (ref_rs = 1).
    constexpr int LDT = 73;
    static_assert(64 * LDT * sizeof(float) <= sizeof(smem), "the output tile must fit the slice buffers");
    float* Ts = reinterpret_cast<float*>(smem);
    __syncthreads();  // every wave is done with the slices
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) Ts[(wm + 16 * i + 4 * quad + r) * LDT + wn + 16 * j + row] = acc[i][j][r];
    __syncthreads();
    for (int q = tid; q < 64 * 8; q += 256) {
      const int c = q & 7, nn = q >> 3;
      const int gm = m0 + 8 * c, gn = n0 + nn;
      if (gm >= g.M || gn >= g.N) continue;
      const bool full = gm + 8 <= g.M;
      const bf16* rp = g.ref + (int64_t)gn * g.ref_cs + gm;
      bf16x8 rv;
      if (full) {
        rv = *reinterpret_cast<const bf16x8*>(rp);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) rv[e] = gm + e < g.M ? rp[e] : (bf16)0.0f;
      }
      bf16x8 t;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        float* tp = Ts + (8 * c + e) * LDT + nn;
        t[e] = (bf16)(*tp * ((float)rv[e] > 0.0f ? 1.0f : SLOPE));
        *tp = (float)t[e];
      }
      bf16* dp = g.CbT + (int64_t)gn * g.ldt + gm;
      if (full) {
        *reinterpret_cast<bf16x8*>(dp) = t;
      } else {
        for (int e = 0; gm + e < g.M; ++e) dp[e] = t[e];
      }
    }
    __syncthreads();
    for (int q = tid; q < 64 * 8; q += 256) {
      const int k = q & 7, mm = q >> 3;
      const int gm = m0 + mm, gn = n0 + 8 * k;
      if (gm >= g.M || gn >= g.N) continue;
      bf16x8 t;
#pragma unroll
      for (int e = 0; e < 8; ++e) t[e] = (bf16)Ts[mm * LDT + 8 * k + e];
      bf16* dp = g.Cb + (int64_t)gm * g.ldc + gn;
      if (gn + 8 <= g.N) {
        *reinterpret_cast<bf16x8*>(dp) = t;
      } else {
        for (int e = 0; gn + e < g.N; ++e) dp[e] = t[e];
      }
    }
  }
}

// out[m ldo + map(n)] = sum_z part[z][m][n] (+ part[z][m + fold][n] when
// fold > 0: the two halves of a split input) for m < m_real, and
// bias[map(n)] = sum_z part[z][M][n] (the column-sum row); partials have
// M + 1 rows.  The column map drops the padding of groups of gpad columns to
// greal (gpad = 0: identity).  Sums run over z in order.
__global__ void k_reduce_grad(const float* __restrict__ part, int Z, int M, int N, int m_real, int gpad, int greal,
                              float* __restrict__ out, int ldo, int fold, float* __restrict__ bias) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)(m_real + 1) * N) return;
  const int m = (int)(idx / N);
  const int nn = (int)(idx % N);
  int col = nn;
  if (gpad) {
    if (nn % gpad >= greal) return;
    col = (nn / gpad) * greal + nn % gpad;
  }
  const int64_t zs = (int64_t)(M + 1) * N;
  if (m == m_real) {
    float s = 0.0f;
    for (int z = 0; z < Z; ++z) s += part[z * zs + (int64_t)M * N + nn];
    bias[col] = s;
    return;
  }
  float s = 0.0f;
  for (int z = 0; z < Z; ++z) {
    s += part[z * zs + (int64_t)m * N + nn];
    if (fold) s += part[z * zs + (int64_t)(m + fold) * N + nn];
  }
  out[(int64_t)m * ldo + col] = s;
}

// g[a_idx[i]][e] += gx[e][i] (gradient reaching the kept coordinates)
__global__ void k_add_gx(LayerDev L, const float* __restrict__ gx, int64_t n, float* __restrict__ g) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * L.dA) return;
  const int i = (int)(idx / n);
  const int64_t e = idx % n;
  g[(int64_t)L.a_idx[i] * n + e] += gx[e * KA + i];
}

// sum of w over the batch (one block, fixed order) and the loss
// -sum w logq / sum w
constexpr int RB = 1024;  // threads of the single-block batch reductions
__global__ void __launch_bounds__(RB) k_wsum(const float* __restrict__ w, int64_t n, float* __restrict__ out) {
  __shared__ double s[RB];
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += RB) a += w[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int st = RB / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)s[0];
}
// variance loss: per-point weights w^2 / q (held fixed in the backward pass)
__global__ void k_variance_weights(const float* __restrict__ w, const float* __restrict__ logq, int64_t n,
                                   float* __restrict__ weff) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) weff[e] = w[e] * w[e] * __expf(-logq[e]);
}
// relative variance per event of sampling q, from points uniform in y:
// n sum w^2/q / (sum w)^2 - 1
__global__ void __launch_bounds__(RB) k_relvar(const float* __restrict__ w, const float* __restrict__ weff, int64_t n,
                                               float* __restrict__ out) {
  __shared__ double s1[RB], s2[RB];
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += RB) {
    a += w[i];
    b += weff[i];
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int st = RB / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      s1[threadIdx.x] += s1[threadIdx.x + st];
      s2[threadIdx.x] += s2[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)((double)n * s2[0] / (s1[0] * s1[0]) - 1.0);
}
__global__ void __launch_bounds__(RB) k_loss(const float* __restrict__ w, const float* __restrict__ logq, int64_t n,
                                             const float* __restrict__ wsum, float* __restrict__ out) {
  __shared__ double s[RB];
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += RB) a += (double)w[i] * logq[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int st = RB / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (float)(-s[0] / wsum[0]);
}

// Parameter segments of one layer in the master layout and the BF16 copies.
struct SegLayer {
  int64_t off;  // start of the layer in the master array
  int dA, dB;
  bf16* W1t;
  float* b3p;
  bf16* W2p;
  bf16* W3p;
  bf16* W3L;
  bf16* W2n;
  bf16* W3n;
};
struct SegTable {
  int nl;
  SegLayer l[MAXL];
};

// Adam on the masters (in place) and refresh of the BF16 copies.  With
// do_adam = 0 only the copies are refreshed.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ gr, float* __restrict__ m1,
                       float* __restrict__ m2, int64_t count, float lr, float c1, float c2, int do_adam, SegTable S) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  float v = p[i];
  if (do_adam) {
    const float gg = gr[i];
    const float a = 0.9f * m1[i] + 0.1f * gg;
    const float b = 0.999f * m2[i] + 0.001f * gg * gg;
    m1[i] = a;
    m2[i] = b;
    v -= lr * (a / c1) / (sqrtf(b / c2) + 1e-8f);
    p[i] = v;
  }
  int l = 0;
  while (l + 1 < S.nl && i >= S.l[l + 1].off) ++l;
  const SegLayer& s = S.l[l];
  int64_t r = i - s.off;
  const int64_t nW1 = (int64_t)s.dA * H, nW2 = (int64_t)H * H, nO = (int64_t)s.dB * NO;
  if (r < nW1) {
    const int a = (int)(r / H), j = (int)(r % H);
    s.W1t[j * KA + a] = (bf16)v;
    s.W1t[j * KA + KLO + a] = (bf16)v;
    return;
  }
  r -= nW1 + H;  // b1 is used in FP32 from the master array
  if (r < 0) return;
  if (r < nW2) {
    const int a = (int)(r / H), j = (int)(r % H);
    s.W2n[r] = (bf16)v;
    // wave j >> 6, fragment (j >> 4) & 3, row j & 15
    s.W2p[(((int64_t)(j >> 6) * 8 + (a >> 5)) * 4 + ((j >> 4) & 3)) * 512 + ((j & 15) + 16 * ((a >> 3) & 3)) * 8 +
          (a & 7)] = (bf16)v;
    return;
  }
  r -= nW2 + H;
  if (r < 0) return;
  if (r < H * nO) {
    const int a = (int)(r / nO), o = (int)(r % nO);
    s.W3n[(int64_t)a * s.dB * NOP + (o / NO) * NOP + o % NO] = (bf16)v;
    const int c = o / NO, col = o % NO;
    // coordinate c, wave col >> 4, row col & 15; the 65th logit in row c of W3L
    if (col < 64)
      s.W3p[(((int64_t)c * 4 + (col >> 4)) * 8 + (a >> 5)) * 512 + ((col & 15) + 16 * ((a >> 3) & 3)) * 8 + (a & 7)] =
          (bf16)v;
    else if (col == 2 * KB)
      s.W3L[((a >> 5) * 64 + c + 16 * ((a >> 3) & 3)) * 8 + (a & 7)] = (bf16)v;
    return;
  }
  r -= H * nO;
  s.b3p[(r / NO) * NOP + r % NO] = v;
}

// Initial parameters: the weights of the first two dense layers of every
// coupling layer uniform in +-sqrt(6 / fan_in) from Philox4x64-10 (counter
// (index, 0, 0, 0), key (seed, 3)); biases and the output layer zero, so the
// flow starts as the identity map while every layer's gradient is live.
__global__ void k_init_params(float* __restrict__ p, int64_t count, uint64_t seed, SegTable S) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  int l = 0;
  while (l + 1 < S.nl && i >= S.l[l + 1].off) ++l;
  const SegLayer& s = S.l[l];
  const int64_t r = i - s.off, nW1 = (int64_t)s.dA * H, nW2 = (int64_t)H * H;
  float a = 0.0f;
  if (r < nW1) a = sqrtf(6.0f / (float)s.dA);
  else if (r >= nW1 + H && r < nW1 + H + nW2) a = sqrtf(6.0f / (float)H);
  float v = 0.0f;
  if (a > 0.0f) {
    const U4 q = philox4x64_10((uint64_t)i, 0, 0, 0, seed, 3);
    v = (float)((2.0 * u01(q.x0) - 1.0) * a);
  }
  p[i] = v;
}

}  // namespace flow
}  // namespace mf

using namespace mf;
using namespace mf::flow;

struct mf_flow {
  mf_flow_config cfg;
  int d, nl;
  int64_t count = 0;
  std::vector<std::vector<uint8_t>> mask;
  LayerDev L[MAXL];
  SegTable seg;
  int64_t loff[MAXL];
  float* d_p = nullptr;   // masters
  float* d_g = nullptr;   // gradient
  float* d_m1 = nullptr;  // Adam moments
  float* d_m2 = nullptr;
  bf16* d_w16 = nullptr;  // BF16 weight copies of every layer
  float* d_b3p = nullptr;
  int64_t step = 0;
  // training caches and work buffers (max_batch events)
  int64_t cap = 0;
  LayerCache cache[MAXL];
  void* d_cachemem = nullptr;
  float* d_y = nullptr;     // [d][cap]
  float* d_gy = nullptr;    // [d][cap]
  float* d_lq = nullptr;    // [cap]
  float* d_weff = nullptr;  // [cap] per-point loss weights of the variance loss
  bf16* d_go = nullptr;     // [cap][dBmax*NOP]
  bf16* d_ga2 = nullptr;    // [cap][H]
  bf16* d_ga1 = nullptr;    // [cap][H]
  bf16* d_goT = nullptr;    // [dBmax*NOP][capp]  event-contiguous copies
  bf16* d_ga2T = nullptr;   // [H][capp]
  bf16* d_ga1T = nullptr;   // [H][capp]
  float* d_gx = nullptr;    // [cap][KA]
  float* d_part = nullptr;  // split-K partials
  size_t part_cap = 0;
  float* d_scal = nullptr;  // wsum, loss
  std::vector<float*> d_losses;
  // the backward pass runs the weight-gradient products on a second stream
  // (default priority) beside the activation-gradient chain; events order
  // the two
  hipStream_t side = nullptr;
  hipEvent_t ev[6] = {};
};

namespace {

constexpr int64_t SPLITK_BLOCKS = 512;
constexpr int64_t SPLITK_MIN = 256;
// at most this many chunks: the ordered reduction sums them sequentially per
// output, which for the narrow first-layer gradient (four output tiles) would
// otherwise take 128 partials
constexpr int64_t SPLITK_MAX = 32;

mf_status launch_err(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(MF_EDEVICE, "%s launch: %s", what, hipGetErrorString(e));
  return MF_OK;
}

template <int A_KC, int B_NC, int EPI>
void gemm(const GemmArgs& a, int Z, hipStream_t s) {
  dim3 grid((a.N + 63) / 64, (a.M + 63) / 64, Z);
  hipLaunchKernelGGL((k_gemm<A_KC, B_NC, EPI>), grid, dim3(256), 0, s, a);
}

// Number of event chunks of a weight-gradient product over n events with an
// M x N output: enough workgroups to fill the chip (about SPLITK_BLOCKS),
// chunks of at least SPLITK_MIN events, at most SPLITK_MAX chunks.
// Non-decreasing in n.
int64_t splitk(int64_t n, int M, int N) {
  const int64_t tiles = (int64_t)((M + 63) / 64) * ((N + 63) / 64);
  int64_t z = (SPLITK_BLOCKS + tiles - 1) / tiles;
  z = z < SPLITK_MAX ? z : SPLITK_MAX;
  const int64_t zmax = (n + SPLITK_MIN - 1) / SPLITK_MIN;
  z = z < zmax ? z : zmax;
  return z < 1 ? 1 : z;
}

// Weight and bias gradients over the batch: dW[in][out] = X^T G and
// db[out] = column sums of G, from the event-contiguous BF16 copies
// XT [M][ldn] and GT [N][ldn], split over events.
bool weight_grad(mf_flow* f, const bf16* XT, int64_t ldn, int M, int m_real, const bf16* GT, int N, int gpad,
                 int greal, int64_t n, float* out, int ldo, float* bias, hipStream_t s, int fold = 0) {
  const int64_t Z = splitk(n, M, N);
  const int64_t chunk = ((n + Z - 1) / Z + 31) / 32 * 32;
  const int Zl = (int)((n + chunk - 1) / chunk);
  // the partials of all chunks must fit the buffer sized at creation
  if ((size_t)Zl * (size_t)(M + 1) * (size_t)N > f->part_cap) return false;
  GemmArgs a{};
  a.A = XT;  // A(m, k) = XT[m ldn + k]
  a.lda = ldn;
  a.B = GT;  // B(k, n) = GT[n ldn + k]
  a.ldb = ldn;
  a.M = M;
  a.N = N;
  a.K = n;
  a.kchunk = chunk;
  a.Cf = f->d_part;
  a.zs = (int64_t)(M + 1) * N;
  a.ldc = N;
  a.colsum = 1;
  gemm<1, 0, 0>(a, Zl, s);
  const int64_t tot = (int64_t)(m_real + 1) * N;
  hipLaunchKernelGGL(k_reduce_grad, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, f->d_part, Zl, M, N, m_real,
                     gpad, greal, out, ldo, fold, bias);
  return true;
}

void run_layers(mf_flow* f, float* y, int64_t n, int64_t ld, float* logq, bool inverse, bool cache, hipStream_t s) {
  const unsigned nblk = (unsigned)((n + T - 1) / T);
  for (int k = 0; k < f->nl; ++k) {
    const int l = inverse ? f->nl - 1 - k : k;
    LayerCache C = cache ? f->cache[l] : LayerCache{};
    if (inverse)
      hipLaunchKernelGGL((k_coupling<true, false>), dim3(nblk), dim3(256), 0, s, f->L[l], y, n, ld, logq,
                         k == 0 ? 1 : 0, C, f->d);
    else if (cache)
      hipLaunchKernelGGL((k_coupling<false, true>), dim3(nblk), dim3(256), 0, s, f->L[l], y, n, ld, logq,
                         k == 0 ? 1 : 0, C, f->d);
    else
      hipLaunchKernelGGL((k_coupling<false, false>), dim3(nblk), dim3(256), 0, s, f->L[l], y, n, ld, logq,
                         k == 0 ? 1 : 0, C, f->d);
  }
}

mf_status refresh(mf_flow* f, hipStream_t s, int do_adam, float lr, float c1, float c2) {
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((f->count + 255) / 256)), dim3(256), 0, s, f->d_p, f->d_g, f->d_m1,
                     f->d_m2, f->count, lr, c1, c2, do_adam, f->seg);
  return launch_err("k_adam");
}

mf_status copy_points(mf_flow* f, const float* src, int64_t n, float* dst, hipStream_t s) {
  if (src == dst) return MF_OK;
  hipError_t e = hipMemcpyAsync(dst, src, sizeof(float) * f->d * n, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return set_error(MF_EDEVICE, "copy of points: %s", hipGetErrorString(e));
  return MF_OK;
}

mf_status loss_grad_impl(mf_flow* f, const float* y, int64_t ldy, const float* w_in, int64_t n, int kind,
                         float* loss_dev, hipStream_t s) {
  const int d = f->d;
  hipError_t e = hipMemcpy2DAsync(f->d_y, sizeof(float) * n, y, sizeof(float) * ldy, sizeof(float) * n, d,
                                  hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return set_error(MF_EDEVICE, "batch copy: %s", hipGetErrorString(e));
  const int64_t ldn = (n + 7) / 8 * 8;
  for (int l = 0; l < f->nl; ++l) f->cache[l].ldn = ldn;
  run_layers(f, f->d_y, n, n, f->d_lq, false, true, s);
  const float* w = w_in;
  if (kind == MF_FLOW_LOSS_VARIANCE) {
    hipLaunchKernelGGL(k_variance_weights, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w_in, f->d_lq, n,
                       f->d_weff);
    w = f->d_weff;
    hipLaunchKernelGGL(k_relvar, dim3(1), dim3(RB), 0, s, w_in, f->d_weff, n, loss_dev);
  }
  hipLaunchKernelGGL(k_wsum, dim3(1), dim3(RB), 0, s, w, n, f->d_scal);
  if (kind != MF_FLOW_LOSS_VARIANCE)
    hipLaunchKernelGGL(k_loss, dim3(1), dim3(RB), 0, s, w, f->d_lq, n, f->d_scal, loss_dev);
  e = hipMemsetAsync(f->d_gy, 0, sizeof(float) * d * n, s);
  if (e != hipSuccess) return set_error(MF_EDEVICE, "gradient clear: %s", hipGetErrorString(e));
  // Per layer the activation-gradient chain (PQ backward, ga2, ga1, gx) runs
  // on s and the three weight-gradient products on the side stream, each
  // started once its input exists on s; before a layer's kernels overwrite
  // go/goT, ga2/ga2T or ga1/ga1T, s waits until the previous layer's product
  // that reads them has run.  All split-K partials are on the side stream.
  hipStream_t s2 = f->side;
  enum { E_PQ, E_GA2, E_GA1, E_W3, E_W2, E_W1 };
  bool ok = true;
  auto rec = [&](int k, hipStream_t from) { ok = ok && hipEventRecord(f->ev[k], from) == hipSuccess; };
  auto wait = [&](int k, hipStream_t on) { ok = ok && hipStreamWaitEvent(on, f->ev[k], 0) == hipSuccess; };
  for (int l = f->nl - 1; l >= 0; --l) {
    const LayerDev& L = f->L[l];
    const LayerCache& C = f->cache[l];
    const int NB = L.dB * NOP, nO = L.dB * NO;
    const bool later = l < f->nl - 1;  // a previous layer's products exist
    float* gW1 = f->d_g + f->loff[l];
    float* gb1 = gW1 + (int64_t)L.dA * H;
    float* gW2 = gb1 + H;
    float* gb2 = gW2 + (int64_t)H * H;
    float* gW3 = gb2 + H;
    float* gb3 = gW3 + (int64_t)H * nO;
    if (later) wait(E_W3, s);
    hipLaunchKernelGGL(k_pq_backward, dim3((unsigned)((n + 255) / 256), L.dB), dim3(256), 0, s, L, C, n, f->d_gy, w,
                       f->d_scal, f->d_go, f->d_goT);
    rec(E_PQ, s);
    wait(E_PQ, s2);
    if (!weight_grad(f, C.h2, ldn, H, H, f->d_goT, NB, NOP, NO, n, gW3, nO, gb3, s2))
      return set_error(MF_EINVAL, "weight-gradient partials exceed the flow's buffer");
    rec(E_W3, s2);
    // ga2 = (go W3^T) * leaky'(h2): A = go [n][NB], B(k=o, n=j) = W3n[j][o]
    GemmArgs a{};
    a.A = f->d_go;
    a.lda = NB;
    a.B = L.W3n;
    a.ldb = NB;
    a.M = (int)n;
    a.N = H;
    a.K = NB;
    a.kchunk = NB;
    a.Cb = f->d_ga2;
    a.CbT = f->d_ga2T;
    a.ldt = ldn;
    a.ref = C.h2;
    a.ref_rs = 1;
    a.ref_cs = ldn;
    a.ldc = H;
    if (later) wait(E_W2, s);
    gemm<1, 0, 1>(a, 1, s);
    rec(E_GA2, s);
    wait(E_GA2, s2);
    if (!weight_grad(f, C.h1, ldn, H, H, f->d_ga2T, H, 0, 0, n, gW2, H, gb2, s2))
      return set_error(MF_EINVAL, "weight-gradient partials exceed the flow's buffer");
    rec(E_W2, s2);
    // ga1 = (ga2 W2^T) * leaky'(h1): B(k=j2, n=j1) = W2[j1][j2] = W2n[j1][j2]
    a.A = f->d_ga2;
    a.lda = H;
    a.B = L.W2n;
    a.ldb = H;
    a.K = H;
    a.kchunk = H;
    a.Cb = f->d_ga1;
    a.CbT = f->d_ga1T;
    a.ref = C.h1;
    if (later) wait(E_W1, s);
    gemm<1, 0, 1>(a, 1, s);
    rec(E_GA1, s);
    wait(E_GA1, s2);
    if (!weight_grad(f, C.xa, ldn, KA, L.dA, f->d_ga1T, H, 0, 0, n, gW1, H, gb1, s2, KLO))
      return set_error(MF_EINVAL, "weight-gradient partials exceed the flow's buffer");
    rec(E_W1, s2);
    // gx = ga1 W1^T: B(k=j, n=i) = W1[i][j] = W1t[j][i]
    GemmArgs b{};
    b.A = f->d_ga1;
    b.lda = H;
    b.B = L.W1t;
    b.ldb = KA;
    b.M = (int)n;
    b.N = KA;
    b.K = H;
    b.kchunk = H;
    b.Cf = f->d_gx;
    b.zs = 0;
    b.ldc = KA;
    gemm<1, 1, 0>(b, 1, s);
    const int64_t ta = n * L.dA;
    if (ta > 0)
      hipLaunchKernelGGL(k_add_gx, dim3((unsigned)((ta + 255) / 256)), dim3(256), 0, s, L, f->d_gx, n, f->d_gy);
  }
  // the gradient is complete on s once the side stream's last product is
  wait(E_W1, s);
  if (!ok) return set_error(MF_EDEVICE, "backward stream ordering failed");
  return launch_err("flow backward");
}

}  // namespace

namespace mf {
mf_status flow_apply(mf_flow* f, float* y, int64_t n, int64_t ld, float* logq, bool inverse, hipStream_t s) {
  if (n <= 0) return MF_OK;
  run_layers(f, y, n, ld, logq, inverse, false, s);
  return launch_err("k_coupling");
}
mf_status flow_step(mf_flow* f, const float* y, int64_t ld, const float* w, int64_t n, float* loss_dev, double lr,
                    hipStream_t s) {
  if (n < 1 || n > f->cap) return set_error(MF_EINVAL, "batch must be in 1..%lld", (long long)f->cap);
  mf_status st = loss_grad_impl(f, y, ld, w, n, MF_FLOW_LOSS_KL, loss_dev, s);
  if (st != MF_OK) return st;
  return mf_flow_adam_step(f, lr, s);
}
}  // namespace mf

extern "C" {

mf_status mf_flow_create(const mf_flow_config* cfg, mf_flow** out) {
  clear_error();
  if (!cfg || !out) return set_error(MF_EINVAL, "NULL argument");
  *out = nullptr;
  if (cfg->ndim < 2 || cfg->ndim > FMAXD) return set_error(MF_EINVAL, "ndim must be in 2..%d", FMAXD);
  static_assert(FMAXD - 1 <= KLO, "kept coordinates must fit the high half of the first-layer inputs");
  if (cfg->n_layers < 1 || cfg->n_layers > MAXL) return set_error(MF_EINVAL, "n_layers must be in 1..%d", MAXL);
  if (cfg->hidden != H) return set_error(MF_ENOTSUP, "only hidden width %d is built", H);
  if (cfg->bins != KB) return set_error(MF_ENOTSUP, "only %d bins are built", KB);
  if (cfg->max_batch < 1 || cfg->max_batch > (1LL << 24))
    return set_error(MF_EINVAL, "max_batch must be in 1..2^24");
  mf_flow* f = new mf_flow();
  f->cfg = *cfg;
  f->d = cfg->ndim;
  f->nl = cfg->n_layers;
  const int d = f->d;
  int nb = 0;
  while ((1 << nb) < d) ++nb;
  if (nb < 1) nb = 1;
  int64_t off = 0, w16 = 0, b3 = 0, dBmax = 0;
  f->seg.nl = f->nl;
  for (int l = 0; l < f->nl; ++l) {
    std::vector<uint8_t> m(d);
    LayerDev& L = f->L[l];
    L.dA = L.dB = 0;
    for (int j = 0; j < d; ++j) {
      const int bit = (j >> (l % nb)) & 1;
      m[j] = (uint8_t)(bit == (((l / nb) % 2 == 0) ? 1 : 0));
      if (m[j]) L.b_idx[L.dB++] = j;
      else L.a_idx[L.dA++] = j;
    }
    f->mask.push_back(m);
    f->loff[l] = off;
    f->seg.l[l].off = off;
    f->seg.l[l].dA = L.dA;
    f->seg.l[l].dB = L.dB;
    off += (int64_t)L.dA * H + H + (int64_t)H * H + H + (int64_t)H * L.dB * NO + L.dB * NO;
    w16 += (int64_t)H * KA + (int64_t)H * H + (int64_t)L.dB * 64 * H + (int64_t)16 * H + (int64_t)H * H +
           (int64_t)H * L.dB * NOP;
    b3 += (int64_t)L.dB * NOP;
    if (L.dB > dBmax) dBmax = L.dB;
  }
  f->count = off;
  auto cleanup = [&](mf_status s) {
    mf_flow_destroy(f);
    return s;
  };
  // the layer kernel keeps the transformed coordinates' inputs in a tile of
  // TBMAX rows (the masks above never transform more than half of 16)
  if (dBmax > TBMAX) return cleanup(set_error(MF_EINVAL, "a layer transforms more than %d coordinates", TBMAX));
  const int64_t cap = cfg->max_batch;
  f->cap = cap;
  // caches: xa, h1, h2, o, lin per layer
  const int64_t capp = (cap + 7) / 8 * 8;
  size_t per_layer = sizeof(bf16) * (size_t)capp * (KA + 2 * H) + sizeof(float) * (size_t)cap * (dBmax * NOP + d);
  per_layer = (per_layer + 255) / 256 * 256;  // every layer's caches start 256-byte aligned
  // the chunk count depends on the output tiles, so a narrower output could
  // need more partials than the widest one: the maximum over every width
  int64_t pc = std::max(splitk(cap, H, H) * (H + 1) * H, splitk(cap, KA, H) * (KA + 1) * H);
  for (int dB = 1; dB <= dBmax; ++dB) pc = std::max(pc, splitk(cap, H, dB * NOP) * (H + 1) * dB * NOP);
  f->part_cap = (size_t)pc;
  if (hipMalloc(&f->d_p, sizeof(float) * off) != hipSuccess || hipMalloc(&f->d_g, sizeof(float) * off) != hipSuccess ||
      hipMalloc(&f->d_m1, sizeof(float) * off) != hipSuccess || hipMalloc(&f->d_m2, sizeof(float) * off) != hipSuccess ||
      hipMalloc(&f->d_w16, sizeof(bf16) * w16) != hipSuccess || hipMalloc(&f->d_b3p, sizeof(float) * b3) != hipSuccess ||
      hipMalloc(&f->d_cachemem, per_layer * f->nl) != hipSuccess ||
      hipMalloc(&f->d_y, sizeof(float) * d * cap) != hipSuccess ||
      hipMalloc(&f->d_gy, sizeof(float) * d * cap) != hipSuccess ||
      hipMalloc(&f->d_lq, sizeof(float) * cap) != hipSuccess ||
      hipMalloc(&f->d_weff, sizeof(float) * cap) != hipSuccess ||
      hipMalloc(&f->d_go, sizeof(bf16) * cap * dBmax * NOP) != hipSuccess ||
      hipMalloc(&f->d_ga2, sizeof(bf16) * cap * H) != hipSuccess ||
      hipMalloc(&f->d_ga1, sizeof(bf16) * cap * H) != hipSuccess ||
      hipMalloc(&f->d_goT, sizeof(bf16) * capp * dBmax * NOP) != hipSuccess ||
      hipMalloc(&f->d_ga2T, sizeof(bf16) * capp * H) != hipSuccess ||
      hipMalloc(&f->d_ga1T, sizeof(bf16) * capp * H) != hipSuccess ||
      hipMalloc(&f->d_gx, sizeof(float) * cap * KA) != hipSuccess ||
      hipMalloc(&f->d_part, sizeof(float) * f->part_cap) != hipSuccess ||
      hipMalloc(&f->d_scal, sizeof(float) * 4) != hipSuccess) {
    hipGetLastError();
    return cleanup(set_error(MF_ENOMEM, "flow allocation failed"));
  }
  if (hipMemset(f->d_g, 0, sizeof(float) * off) != hipSuccess ||
      hipMemset(f->d_m1, 0, sizeof(float) * off) != hipSuccess ||
      hipMemset(f->d_m2, 0, sizeof(float) * off) != hipSuccess ||
      hipMemset(f->d_w16, 0, sizeof(bf16) * w16) != hipSuccess ||
      hipMemset(f->d_b3p, 0, sizeof(float) * b3) != hipSuccess)
    return cleanup(set_error(MF_EDEVICE, "flow initialisation failed"));
  if (hipStreamCreateWithFlags(&f->side, hipStreamNonBlocking) != hipSuccess) {
    f->side = nullptr;
    hipGetLastError();
    return cleanup(set_error(MF_EDEVICE, "flow stream creation failed"));
  }
  for (hipEvent_t& e : f->ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      e = nullptr;
      hipGetLastError();
      return cleanup(set_error(MF_EDEVICE, "flow event creation failed"));
    }
  bf16* wp = f->d_w16;
  float* bp = f->d_b3p;
  char* cm = (char*)f->d_cachemem;
  for (int l = 0; l < f->nl; ++l) {
    LayerDev& L = f->L[l];
    L.W1t = wp;
    f->seg.l[l].W1t = wp;
    wp += (int64_t)H * KA;
    L.W2p = wp;
    f->seg.l[l].W2p = wp;
    wp += (int64_t)H * H;
    L.W3p = wp;
    f->seg.l[l].W3p = wp;
    wp += (int64_t)L.dB * 64 * H;
    L.W3L = wp;
    f->seg.l[l].W3L = wp;
    wp += (int64_t)16 * H;
    L.W2n = wp;
    f->seg.l[l].W2n = wp;
    wp += (int64_t)H * H;
    L.W3n = wp;
    f->seg.l[l].W3n = wp;
    wp += (int64_t)H * L.dB * NOP;
    L.b3p = bp;
    f->seg.l[l].b3p = bp;
    bp += (int64_t)L.dB * NOP;
    L.b1 = f->d_p + f->loff[l] + (int64_t)L.dA * H;
    L.b2 = L.b1 + H + (int64_t)H * H;
    LayerCache& C = f->cache[l];
    C.xa = (bf16*)cm;
    cm += sizeof(bf16) * capp * KA;
    C.h1 = (bf16*)cm;
    cm += sizeof(bf16) * capp * H;
    C.h2 = (bf16*)cm;
    cm += sizeof(bf16) * capp * H;
    C.ldn = capp;
    C.o = (float*)cm;
    cm += sizeof(float) * cap * dBmax * NOP;
    C.lin = (float*)cm;
    cm = (char*)f->d_cachemem + per_layer * (size_t)(l + 1);
  }
  hipLaunchKernelGGL(k_init_params, dim3((unsigned)((off + 255) / 256)), dim3(256), 0, 0, f->d_p, off, cfg->seed,
                     f->seg);
  if (refresh(f, nullptr, 0, 0.0f, 1.0f, 1.0f) != MF_OK || hipDeviceSynchronize() != hipSuccess)
    return cleanup(set_error(MF_EDEVICE, "flow parameter initialisation failed"));
  *out = f;
  return MF_OK;
}

void mf_flow_destroy(mf_flow* f) {
  if (!f) return;
  hipFree(f->d_p);
  hipFree(f->d_g);
  hipFree(f->d_m1);
  hipFree(f->d_m2);
  hipFree(f->d_w16);
  hipFree(f->d_b3p);
  hipFree(f->d_cachemem);
  hipFree(f->d_y);
  hipFree(f->d_gy);
  hipFree(f->d_lq);
  hipFree(f->d_weff);
  hipFree(f->d_go);
  hipFree(f->d_ga2);
  hipFree(f->d_ga1);
  hipFree(f->d_goT);
  hipFree(f->d_ga2T);
  hipFree(f->d_ga1T);
  hipFree(f->d_gx);
  hipFree(f->d_part);
  hipFree(f->d_scal);
  for (float* p : f->d_losses) hipFree(p);
  for (hipEvent_t e : f->ev)
    if (e) hipEventDestroy(e);
  if (f->side) hipStreamDestroy(f->side);
  delete f;
}

int64_t mf_flow_param_count(const mf_flow* f) { return f ? f->count : -1; }

int mf_flow_ndim(const mf_flow* f) { return f ? f->d : 0; }

mf_status mf_flow_masks(const mf_flow* f, uint8_t* out) {
  clear_error();
  if (!f || !out) return set_error(MF_EINVAL, "NULL argument");
  for (int l = 0; l < f->nl; ++l) std::memcpy(out + (size_t)l * f->d, f->mask[l].data(), f->d);
  return MF_OK;
}

mf_status mf_flow_set_params(mf_flow* f, const float* params, int64_t count) {
  clear_error();
  if (!f || !params) return set_error(MF_EINVAL, "NULL argument");
  if (count != f->count) return set_error(MF_EINVAL, "expected %lld parameters, got %lld", (long long)f->count,
                                          (long long)count);
  if (hipMemcpy(f->d_p, params, sizeof(float) * count, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(f->d_m1, 0, sizeof(float) * count) != hipSuccess ||
      hipMemset(f->d_m2, 0, sizeof(float) * count) != hipSuccess)
    return set_error(MF_EDEVICE, "parameter upload failed");
  f->step = 0;
  mf_status st = refresh(f, nullptr, 0, 0.0f, 1.0f, 1.0f);
  if (st != MF_OK) return st;
  if (hipDeviceSynchronize() != hipSuccess) return set_error(MF_EDEVICE, "parameter refresh failed");
  return MF_OK;
}

mf_status mf_flow_get_params(const mf_flow* f, float* params, int64_t count) {
  clear_error();
  if (!f || !params) return set_error(MF_EINVAL, "NULL argument");
  if (count != f->count) return set_error(MF_EINVAL, "expected %lld parameters", (long long)f->count);
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(params, f->d_p, sizeof(float) * count, hipMemcpyDeviceToHost) != hipSuccess)
    return set_error(MF_EDEVICE, "parameter download failed");
  return MF_OK;
}

mf_status mf_flow_forward(mf_flow* f, const float* y, int64_t n, float* z, float* logq, void* stream) {
  clear_error();
  if (!f) return set_error(MF_EINVAL, "NULL flow");
  if (n < 0) return set_error(MF_EINVAL, "negative event count");
  if (n == 0) return MF_OK;
  if (!y || !z || !logq) return set_error(MF_EINVAL, "NULL buffer");
  hipStream_t s = (hipStream_t)stream;
  mf_status st = copy_points(f, y, n, z, s);
  if (st != MF_OK) return st;
  run_layers(f, z, n, n, logq, false, false, s);
  return launch_err("k_coupling");
}

mf_status mf_flow_inverse(mf_flow* f, const float* z, int64_t n, float* y, float* logq, void* stream) {
  clear_error();
  if (!f) return set_error(MF_EINVAL, "NULL flow");
  if (n < 0) return set_error(MF_EINVAL, "negative event count");
  if (n == 0) return MF_OK;
  if (!y || !z || !logq) return set_error(MF_EINVAL, "NULL buffer");
  hipStream_t s = (hipStream_t)stream;
  mf_status st = copy_points(f, z, n, y, s);
  if (st != MF_OK) return st;
  run_layers(f, y, n, n, logq, true, false, s);
  return launch_err("k_coupling");
}

mf_status mf_flow_loss_grad(mf_flow* f, const float* y, const float* w, int64_t n, int32_t loss_kind, float* grad,
                            double* loss, void* stream) {
  clear_error();
  if (!f) return set_error(MF_EINVAL, "NULL flow");
  if (n < 1 || n > f->cap) return set_error(MF_EINVAL, "n must be in 1..%lld", (long long)f->cap);
  if (!y || !w) return set_error(MF_EINVAL, "NULL buffer");
  if (loss_kind != MF_FLOW_LOSS_KL && loss_kind != MF_FLOW_LOSS_VARIANCE)
    return set_error(MF_EINVAL, "unknown loss %d", loss_kind);
  hipStream_t s = (hipStream_t)stream;
  mf_status st = loss_grad_impl(f, y, n, w, n, loss_kind, f->d_scal + 1, s);
  if (st != MF_OK) return st;
  if (grad && hipMemcpyAsync(grad, f->d_g, sizeof(float) * f->count, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return set_error(MF_EDEVICE, "gradient copy failed");
  if (loss) {
    float l = 0.0f;
    if (hipMemcpyAsync(&l, f->d_scal + 1, sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return set_error(MF_EDEVICE, "loss copy failed");
    *loss = l;
  }
  return MF_OK;
}

mf_status mf_flow_adam_step(mf_flow* f, double lr, void* stream) {
  clear_error();
  if (!f) return set_error(MF_EINVAL, "NULL flow");
  if (!(lr >= 0.0)) return set_error(MF_EINVAL, "learning rate must be >= 0");
  f->step += 1;
  const float c1 = (float)(1.0 - std::pow(0.9, (double)f->step));
  const float c2 = (float)(1.0 - std::pow(0.999, (double)f->step));
  return refresh(f, (hipStream_t)stream, 1, (float)lr, c1, c2);
}

mf_status mf_flow_train(mf_flow* f, const float* y, const float* w, int64_t n, const mf_flow_train_opts* o,
                        double* loss_per_epoch) {
  clear_error();
  if (!f || !o) return set_error(MF_EINVAL, "NULL argument");
  if (!y || !w) return set_error(MF_EINVAL, "NULL buffer");
  if (o->epochs < 1) return set_error(MF_EINVAL, "epochs must be >= 1");
  if (o->batch < 1 || o->batch > f->cap) return set_error(MF_EINVAL, "batch must be in 1..%lld", (long long)f->cap);
  if (n < 1) return set_error(MF_EINVAL, "no training points");
  if (!(o->lr > 0.0) || !(o->lr_final >= 0.0)) return set_error(MF_EINVAL, "invalid learning rates");
  if (o->loss != MF_FLOW_LOSS_KL && o->loss != MF_FLOW_LOSS_VARIANCE)
    return set_error(MF_EINVAL, "unknown loss %d", o->loss);
  hipStream_t s = (hipStream_t)o->stream;
  const int64_t per_epoch = (n + o->batch - 1) / o->batch;
  const int64_t total = per_epoch * o->epochs;
  float* d_loss = nullptr;
  if (hipMalloc(&d_loss, sizeof(float) * total) != hipSuccess) return set_error(MF_ENOMEM, "loss history");
  struct Free {
    float* p;
    ~Free() { (void)hipFree(p); }
  } guard{d_loss};
  int64_t t = 0;
  for (int ep = 0; ep < o->epochs; ++ep) {
    for (int64_t b = 0; b < per_epoch; ++b, ++t) {
      const int64_t off = b * o->batch;
      const int64_t nb = std::min<int64_t>(o->batch, n - off);
      // batch slice of the [d][n] points: rows of nb values with pitch n
      mf_status st = loss_grad_impl(f, y + off, n, w + off, nb, o->loss, d_loss + t, s);
      if (st != MF_OK) return st;
      const double lr = o->lr_final + 0.5 * (o->lr - o->lr_final) * (1.0 + std::cos(M_PI * (double)t / (double)total));
      st = mf_flow_adam_step(f, lr, s);
      if (st != MF_OK) return st;
    }
  }
  std::vector<float> hl((size_t)total);
  if (hipMemcpyAsync(hl.data(), d_loss, sizeof(float) * total, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(MF_EDEVICE, "training failed");
  if (loss_per_epoch)
    for (int ep = 0; ep < o->epochs; ++ep) {
      double a = 0.0;
      for (int64_t b = 0; b < per_epoch; ++b) a += hl[(size_t)(ep * per_epoch + b)];
      loss_per_epoch[ep] = a / (double)per_epoch;
    }
  return MF_OK;
}

}  // extern "C"
