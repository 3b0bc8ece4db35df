// Omnidirectional feature front end (Section 3): the magnitude of the
// discrete Fourier transform of 1-D panoramic signals, bins 0 .. d-1, is the
// rotation-invariant feature the database and the queries hold.
//
// Everything is computed in FP64 and rounded once to fp32. One wave owns one
// signal at a time (64-thread blocks, grid-stride over the signals):
//   * the real signal of length L = 2n is read as n complex points
//     z_t = x_{2t} + i x_{2t+1} (one 8-byte load per lane and point, a wave
//     reads 512 contiguous bytes per instruction) and stored to LDS in
//     bit-reversed order;
//   * an iterative radix-2 decimation-in-time transform of length n runs in
//     LDS, twiddles exp(-i pi j / n) tabulated once per block with sincospi;
//   * the half-length spectrum is unpacked into the spectrum of x,
//     X_j = E_j + exp(-i pi j / n) O_j, with E_j = (Z_j + conj Z_{n-j}) / 2
//     and O_j = (Z_j - conj Z_{n-j}) / 2i the transforms of the even and odd
//     samples, and |X_j| is written (a wave writes 256 contiguous bytes per
//     instruction).
// The kernel reads 4L and writes 4d bytes per signal and does about
// 5 n log2 n + 20 d FP64 operations, so it is bound by HBM.
#include <cmath>

#include "hloc_host.h"

namespace hloc {

constexpr int kFftMaxLen = 2048;   // LDS per block (2n + 1) * 16 bytes <= 32 KB
constexpr int kFftBlocksPerCu = 32;  // one wave each; 8 waves per SIMD at 45 VGPRs

__global__ __launch_bounds__(64) void k_fft_magnitude(const float *__restrict__ x, int64_t nsig,
                                                      int len, int log2n, int d,
                                                      float *__restrict__ out) {
  extern __shared__ double2 lds[];
  const int n = len >> 1;
  double2 *tw = lds;           // tw[j] = exp(-i pi j / n), j = 0 .. n
  double2 *a = lds + (n + 1);  // the length-n transform, in place
  const int lane = threadIdx.x;
  for (int j = lane; j <= n; j += 64) {
    double s, c;
    sincospi((double)j / (double)n, &s, &c);
    tw[j] = make_double2(c, -s);
  }
  for (int64_t sig = blockIdx.x; sig < nsig; sig += gridDim.x) {
    const float2 *row = reinterpret_cast<const float2 *>(x + sig * len);
    __syncthreads();  // the twiddles are written; the previous signal is read out
    for (int t = lane; t < n; t += 64) {
      const float2 v = row[t];
      const int r = log2n ? (int)(__builtin_bitreverse32((uint32_t)t) >> (32 - log2n)) : 0;
      a[r] = make_double2((double)v.x, (double)v.y);
    }
    for (int h = 1; h < n; h <<= 1) {
      __syncthreads();
      const int stride = n / h;  // exp(-2 pi i pos / 2h) = tw[pos * n / h]
      for (int b = lane; b < (n >> 1); b += 64) {
        const int pos = b & (h - 1);
        const int i = ((b - pos) << 1) + pos;
        const double2 w = tw[pos * stride];
        const double2 u = a[i], v = a[i + h];
        const double tr = w.x * v.x - w.y * v.y;
        const double ti = w.x * v.y + w.y * v.x;
        a[i] = make_double2(u.x + tr, u.y + ti);
        a[i + h] = make_double2(u.x - tr, u.y - ti);
      }
    }
    __syncthreads();
    float *o = out + sig * d;
    for (int j = lane; j < d; j += 64) {
      const double2 A = a[j & (n - 1)];        // Z_j (Z_n = Z_0)
      const double2 B = a[(n - j) & (n - 1)];  // Z_{n-j}
      const double er = 0.5 * (A.x + B.x), ei = 0.5 * (A.y - B.y);  // E_j
      const double orr = 0.5 * (A.y + B.y), oi = -0.5 * (A.x - B.x);  // O_j
      const double2 w = tw[j];
      const double xr = er + (w.x * orr - w.y * oi);
      const double xi = ei + (w.x * oi + w.y * orr);
      o[j] = (float)sqrt(xr * xr + xi * xi);
    }
  }
}

}  // namespace hloc

using namespace hloc;

extern "C" int hloc_fft_features_async(const float *signals, int64_t nsig, int32_t len, int32_t d,
                                       float *out, void *stream) {
  if (nsig < 0) return fail(HLOC_EINVAL, "nsig must be >= 0 (got %lld)", (long long)nsig);
  if (len < 2 || len > kFftMaxLen || (len & (len - 1)) != 0)
    return fail(HLOC_EINVAL, "len must be a power of two in 2..%d (got %d)", kFftMaxLen, len);
  if (d < 1 || d > len / 2 + 1)
    return fail(HLOC_EINVAL, "d must be in 1..%d for len %d (got %d)", len / 2 + 1, len, d);
  if (nsig == 0) return HLOC_OK;
  if (!signals || !out) return fail(HLOC_EINVAL, "signals and out must not be NULL");
  int dev = 0, num_cu = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, dev));
  const int n = len / 2;
  const uint32_t lds = (uint32_t)(2 * n + 1) * sizeof(double2);
  const int per_cu = std::max(1, std::min<int>(kFftBlocksPerCu, kLdsPerCu / (int)lds));
  const int64_t grid = std::min<int64_t>(nsig, (int64_t)std::max(num_cu, 1) * per_cu);
  int log2n = 0;
  while ((1 << log2n) < n) ++log2n;
  HIPCHK(launch_kernel(k_fft_magnitude, dim3((unsigned)grid), dim3(64), lds,
                       reinterpret_cast<hipStream_t>(stream), signals, nsig, (int)len, log2n,
                       (int)d, out));
  return HLOC_OK;
}
