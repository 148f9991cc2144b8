// Weight statistics for the unweighting efficiency of a sample: mean,
// maximum, non-zero count (ordered block reductions) and an exact quantile by
// radix selection over order-preserving 64-bit keys of the FP64 weights
// (sign bit flipped for non-negative values, all bits flipped for negative
// ones, so that the unsigned keys sort like the values).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#include "../../include/mf.h"
#include "status.h"

namespace {

constexpr int SB = 256;
constexpr int SMAXB = 1024;

// per-block sum and sum of squares (in a fixed order), max, non-zero and
// invalid counts
constexpr int NS = 5;
__global__ void __launch_bounds__(SB) k_wstat_partial(const double* __restrict__ w, int64_t n, double* __restrict__ part) {
  __shared__ double ss[SB], sm[SB], sz[SB], sb[SB], sq[SB];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per, b1 = b0 + per < n ? b0 + per : n;
  double s = 0.0, m = -INFINITY, z = 0.0, bad = 0.0, q = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += SB) {
    const double v = w[i];
    if (isnan(v)) {
      bad += 1.0;
      continue;
    }
    s += v;
    q += v * v;
    m = v > m ? v : m;
    z += v != 0.0 ? 1.0 : 0.0;
  }
  ss[threadIdx.x] = s;
  sm[threadIdx.x] = m;
  sz[threadIdx.x] = z;
  sb[threadIdx.x] = bad;
  sq[threadIdx.x] = q;
  __syncthreads();
  for (int st = SB / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      ss[threadIdx.x] += ss[threadIdx.x + st];
      sq[threadIdx.x] += sq[threadIdx.x + st];
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + st]);
      sz[threadIdx.x] += sz[threadIdx.x + st];
      sb[threadIdx.x] += sb[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[NS * blockIdx.x + 0] = ss[0];
    part[NS * blockIdx.x + 1] = sm[0];
    part[NS * blockIdx.x + 2] = sz[0];
    part[NS * blockIdx.x + 3] = sb[0];
    part[NS * blockIdx.x + 4] = sq[0];
  }
}

__global__ void k_wstat_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double s = 0.0, m = -INFINITY, z = 0.0, bad = 0.0, q = 0.0;
  for (int b = 0; b < nb; ++b) {
    s += part[NS * b];
    m = fmax(m, part[NS * b + 1]);
    z += part[NS * b + 2];
    bad += part[NS * b + 3];
    q += part[NS * b + 4];
  }
  out[0] = s;
  out[1] = m;
  out[2] = z;
  out[3] = bad;
  out[4] = q;
}

// state: [0] prefix, [1] mask of the fixed high bits, [2] rank still to find
__global__ void k_zero_hist(unsigned long long* hist) {
  if (threadIdx.x < 256) hist[threadIdx.x] = 0ull;
}

__device__ __forceinline__ unsigned long long order_key(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__global__ void __launch_bounds__(SB) k_radix_hist(const double* __restrict__ w, int64_t n,
                                                   const unsigned long long* __restrict__ state, int shift,
                                                   unsigned long long* __restrict__ hist) {
  __shared__ unsigned int h[256];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const unsigned long long prefix = state[0], mask = state[1];
  for (int64_t i = (int64_t)blockIdx.x * SB + threadIdx.x; i < n; i += (int64_t)gridDim.x * SB) {
    const unsigned long long key = order_key(w[i]);
    if ((key & mask) == prefix) atomicAdd(&h[(key >> shift) & 255ull], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

__global__ void k_radix_pick(const unsigned long long* __restrict__ hist, unsigned long long* state, int shift) {
  if (threadIdx.x != 0) return;
  unsigned long long k = state[2], below = 0ull;
  int dsel = 255;
  for (int dg = 0; dg < 256; ++dg) {
    if (below + hist[dg] > k) {
      dsel = dg;
      break;
    }
    below += hist[dg];
  }
  state[0] |= (unsigned long long)dsel << shift;
  state[1] |= 255ull << shift;
  state[2] = k - below;
}

// out[k] = sum_e dw[k][e] g[e]: per-block partial sums in a fixed order, then
// one block adds the partials in order.
__global__ void __launch_bounds__(SB) k_vjp_partial(const double* __restrict__ dw, int k, const double* __restrict__ g,
                                                   int64_t n, double* __restrict__ part) {
  __shared__ double sh[SB];
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = (int64_t)blockIdx.x * per, b1 = b0 + per < n ? b0 + per : n;
  for (int r = 0; r < k; ++r) {
    double a = 0.0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += SB) a += dw[(int64_t)r * n + i] * g[i];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int st = SB / 2; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * k + r] = sh[0];
    __syncthreads();
  }
}
__global__ void k_vjp_final(const double* __restrict__ part, int nb, int k, double* __restrict__ out) {
  const int r = threadIdx.x;
  if (r >= k) return;
  double a = 0.0;
  for (int b = 0; b < nb; ++b) a += part[(int64_t)b * k + r];
  out[r] = a;
}

}  // namespace

// Blocks of the partial-sum kernels for n events.
static int stat_blocks(int64_t n) { return (int)(n < (int64_t)SMAXB * SB ? (n + SB - 1) / SB : SMAXB); }

extern "C" int64_t mf_vjp_workspace(int32_t k, int64_t n) {
  if (k < 1 || n < 1) return 0;
  return (int64_t)sizeof(double) * stat_blocks(n) * k;
}

extern "C" mf_status mf_vjp(const double* dw, int32_t k, const double* g, int64_t n, double* out, void* work,
                            int64_t work_bytes, void* stream) {
  mf::clear_error();
  if (!dw || !g || !out || !work) return mf::set_error(MF_EINVAL, "NULL argument");
  if (k < 1 || k > 64) return mf::set_error(MF_EINVAL, "k must be in 1..64");
  if (n < 1) return mf::set_error(MF_EINVAL, "n must be >= 1");
  if (work_bytes < mf_vjp_workspace(k, n))
    return mf::set_error(MF_EINVAL, "workspace of %lld bytes, %lld needed", (long long)work_bytes,
                         (long long)mf_vjp_workspace(k, n));
  if (((uintptr_t)work & 7) != 0) return mf::set_error(MF_EINVAL, "workspace not 8-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  const int nb = stat_blocks(n);
  double* part = static_cast<double*>(work);
  hipLaunchKernelGGL(k_vjp_partial, dim3(nb), dim3(SB), 0, s, dw, k, g, n, part);
  hipLaunchKernelGGL(k_vjp_final, dim3(1), dim3(64), 0, s, part, nb, k, out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return mf::set_error(MF_EDEVICE, "vjp launch: %s", hipGetErrorString(e));
  return MF_OK;
}

extern "C" int64_t mf_weight_stats_workspace(int64_t n) {
  if (n < 1) return 0;
  // partial sums (NS per block and NS for the total), then the radix state
  return (int64_t)sizeof(double) * (NS * stat_blocks(n) + NS) + (int64_t)sizeof(unsigned long long) * (256 + 3);
}

extern "C" mf_status mf_weight_stats(const double* w, int64_t n, double q, double* out, void* work,
                                     int64_t work_bytes, void* stream) {
  mf::clear_error();
  if (!w || !out || !work) return mf::set_error(MF_EINVAL, "NULL argument");
  if (n < 1) return mf::set_error(MF_EINVAL, "n must be >= 1");
  if (!(q > 0.0 && q <= 1.0)) return mf::set_error(MF_EINVAL, "q must be in (0,1]");
  if (work_bytes < mf_weight_stats_workspace(n))
    return mf::set_error(MF_EINVAL, "workspace of %lld bytes, %lld needed", (long long)work_bytes,
                         (long long)mf_weight_stats_workspace(n));
  if (((uintptr_t)work & 7) != 0) return mf::set_error(MF_EINVAL, "workspace not 8-byte aligned");
  hipStream_t s = (hipStream_t)stream;
  const int nb = stat_blocks(n);
  double* part = static_cast<double*>(work);
  unsigned long long* st = reinterpret_cast<unsigned long long*>(part + NS * nb + NS);
  hipLaunchKernelGGL(k_wstat_partial, dim3(nb), dim3(SB), 0, s, w, n, part);
  hipLaunchKernelGGL(k_wstat_final, dim3(1), dim3(64), 0, s, part, nb, part + NS * nb);
  // rank of the quantile: ceil(q n) - 1
  unsigned long long rank = (unsigned long long)std::ceil(q * (double)n);
  if (rank < 1) rank = 1;
  if (rank > (unsigned long long)n) rank = (unsigned long long)n;
  unsigned long long init[3] = {0ull, 0ull, rank - 1};
  unsigned long long* hist = st + 3;
  mf_status ret = MF_OK;
  if (hipMemcpyAsync(st, init, sizeof(init), hipMemcpyHostToDevice, s) != hipSuccess) ret = MF_EDEVICE;
  for (int shift = 56; shift >= 0 && ret == MF_OK; shift -= 8) {
    hipLaunchKernelGGL(k_zero_hist, dim3(1), dim3(256), 0, s, hist);
    hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(SB), 0, s, w, n, st, shift, hist);
    hipLaunchKernelGGL(k_radix_pick, dim3(1), dim3(64), 0, s, hist, st, shift);
  }
  double tot[NS] = {0, 0, 0, 0, 0};
  unsigned long long res[3] = {0, 0, 0};
  if (ret == MF_OK && (hipGetLastError() != hipSuccess ||
                       hipMemcpyAsync(tot, part + NS * nb, sizeof(tot), hipMemcpyDeviceToHost, s) != hipSuccess ||
                       hipMemcpyAsync(res, st, sizeof(res), hipMemcpyDeviceToHost, s) != hipSuccess ||
                       hipStreamSynchronize(s) != hipSuccess))
    ret = MF_EDEVICE;
  (void)hipStreamSynchronize(s);
  if (ret != MF_OK) return mf::set_error(ret, "weight statistics failed on the device");
  if (tot[3] > 0.0) return mf::set_error(MF_EINVAL, "%.0f weights are NaN", tot[3]);
  out[0] = tot[0] / (double)n;
  out[1] = tot[1];
  double qv;
  const unsigned long long key = res[0];
  unsigned long long bits = (key >> 63) ? (key & 0x7FFFFFFFFFFFFFFFull) : ~key;
  std::memcpy(&qv, &bits, sizeof(qv));
  out[2] = qv;
  out[3] = tot[2];
  const double m1 = tot[0] / (double)n, m2 = tot[4] / (double)n;
  out[4] = m1 != 0.0 ? m2 / (m1 * m1) - 1.0 : 0.0;
  return MF_OK;
}
