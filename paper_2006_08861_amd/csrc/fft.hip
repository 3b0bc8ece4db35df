// Omnidirectional feature front end (Section 3): the magnitude of the
// discrete Fourier transform of 1-D panoramic signals, bins 0 .. d-1, is the
// rotation-invariant feature the database and the queries hold.
//
// Everything is computed in FP64 and rounded once to fp32. The real signal
// of length L = 2n is read as n complex points z_t = x_{2t} + i x_{2t+1},
// transformed at length n, and unpacked into the spectrum of x:
// X_j = E_j + exp(-i pi j / n) O_j, with E_j = (Z_j + conj Z_{n-j}) / 2 and
// O_j = (Z_j - conj Z_{n-j}) / 2i the transforms of the even and odd samples.
// The twiddles exp(-i pi j / n), j = 0 .. n, are tabulated in LDS once per
// block with sincospi.
//
// n = R^2 with R = 8 or 16 (L = 128, 512): four-step transform, R lanes per
// signal and 64 / R signals per wave. Lane c loads points R t1 + c (R lanes
// read 8R contiguous bytes per instruction), transforms them over t1 in
// registers, multiplies by exp(-2 pi i k1 c / n), and the wave transposes its
// signals through padded LDS rows (real parts, then imaginary parts: half the
// LDS of a complex transpose, more blocks per compute unit); lane c then transforms row k1 = c over t2
// in registers and holds Z_{c + R k2}. The partner Z_{n-j} of its bin
// j = c + R k2 sits in lane R - c (lane 0: its own registers) and comes by a
// lane shuffle. The next signals' points are loaded while the current ones
// are transformed. Any other n: one wave per signal, iterative radix-2
// transform in LDS.
//
// Both read 4L and write 4d bytes per signal and do about 5 n log2 n + 20 d
// FP64 operations.
#include <cmath>

#include "hloc_host.h"

namespace hloc {

constexpr int kFftMaxLen = 2048;   // LDS per block (2n + 1) * 16 bytes <= 32 KB
constexpr int kFftBlocksPerCu = 32;  // one wave each; 8 waves per SIMD at 45 VGPRs

constexpr int bit_reverse(int t, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r |= ((t >> i) & 1) << (bits - 1 - i);
  return r;
}

__device__ __forceinline__ double2 cmul(double2 w, double2 v) {
  return make_double2(w.x * v.x - w.y * v.y, w.x * v.y + w.y * v.x);
}

// exp(-2 pi i k / 16), k = 0 .. 7, from cos(pi/8) = sqrt(2 + sqrt 2) / 2,
// sin(pi/8) = sqrt(2 - sqrt 2) / 2 and cos(pi/4) = sqrt(2) / 2 (40 digits,
// rounded to double by the compiler).
constexpr double kC8 = 0.9238795325112867561281831893967882868225;
constexpr double kS8 = 0.3826834323650897717284599840303988667612;
constexpr double kH2 = 0.7071067811865475244008443621048490392848;
__device__ constexpr double w16_re(int k) {
  return k == 0 ? 1.0 : k == 1 ? kC8 : k == 2 ? kH2 : k == 3 ? kS8 : k == 4 ? 0.0
       : k == 5 ? -kS8 : k == 6 ? -kH2 : -kC8;
}
__device__ constexpr double w16_im(int k) {
  return k == 0 ? 0.0 : k == 1 ? -kS8 : k == 2 ? -kH2 : k == 3 ? -kC8 : k == 4 ? -1.0
       : k == 5 ? -kC8 : k == 6 ? -kH2 : -kS8;
}

// In-register transform of length R = 8 or 16 (bit-reversed input, natural
// output), radix-2 decimation in time with compile-time twiddles; the
// twiddles 1 and -i cost no multiply.
template <int R>
__device__ __forceinline__ void dft_regs(double2 (&a)[R]) {
#pragma unroll
  for (int h = 1; h < R; h <<= 1) {
#pragma unroll
    for (int b = 0; b < R / 2; ++b) {
      const int pos = b & (h - 1);
      const int i = ((b - pos) << 1) + pos;
      const int k = pos * (16 / (2 * h));  // exp(-2 pi i pos / 2h) = w16(k)
      double2 v = a[i + h];
      if (k == 4)
        v = make_double2(v.y, -v.x);
      else if (k != 0)
        v = cmul(make_double2(w16_re(k), w16_im(k)), v);
      const double2 u = a[i];
      a[i] = make_double2(u.x + v.x, u.y + v.y);
      a[i + h] = make_double2(u.x - v.x, u.y - v.y);
    }
  }
}

// |X_j| from Z_j (A), Z_{n-j} (B) and tw[j], computed as |2 X_j| / 2 from
// 2 E_j and 2 O_j (scaling by powers of two is exact, so the result is the
// same as with the halvings applied first).
__device__ __forceinline__ float unpack_mag(double2 A, double2 B, double2 w) {
  const double er = A.x + B.x, ei = A.y - B.y;    // 2 E_j
  const double orr = A.y + B.y, oi = B.x - A.x;   // 2 O_j
  const double xr = er + (w.x * orr - w.y * oi);
  const double xi = ei + (w.x * oi + w.y * orr);
  return (float)(0.5 * sqrt(xr * xr + xi * xi));
}

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
      o[j] = unpack_mag(a[j & (n - 1)], a[(n - j) & (n - 1)], tw[j]);  // Z_j, Z_{n-j}
    }
  }
}

template <int R>
constexpr uint32_t fft_sq_lds_bytes() {
  return (uint32_t)((R * R + 1) * sizeof(double2) + (64 / R) * R * (R + 1) * sizeof(double));
}

template <int R>
__global__ __launch_bounds__(64) void k_fft_magnitude_sq(const float *__restrict__ x,
                                                         int64_t nsig, int d,
                                                         float *__restrict__ out) {
  constexpr int N = R * R, G = 64 / R;
  constexpr int LG = R == 8 ? 3 : R == 16 ? 4 : 5;
  static_assert((1 << LG) == R, "R must be 8, 16 or 32");
  extern __shared__ double2 lds[];
  double2 *tw = lds;  // tw[j] = exp(-i pi j / N), j = 0 .. N
  const int lane = threadIdx.x, g = lane / R, c = lane % R;
  // this signal's R x (R + 1) rows (real parts, then imaginary parts)
  double *rows = reinterpret_cast<double *>(lds + (N + 1)) + g * R * (R + 1);
  for (int j = lane; j <= N; j += 64) {
    double sn, cs;
    sincospi((double)j / (double)N, &sn, &cs);
    tw[j] = make_double2(cs, -sn);
  }
  const int64_t stride = (int64_t)gridDim.x * G;
  float2 cur[R];
  {
    const int64_t s = (int64_t)blockIdx.x * G + g;
    const float2 *p = reinterpret_cast<const float2 *>(x) + s * N + c;
#pragma unroll
    for (int t = 0; t < R; ++t) cur[t] = s < nsig ? p[t * R] : make_float2(0.f, 0.f);
  }
  __syncthreads();  // the twiddles are written
  for (int64_t base = (int64_t)blockIdx.x * G; base < nsig; base += stride) {
    const int64_t s = base + g;
    float2 nxt[R];
    {
      const int64_t sn = s + stride;
      const float2 *p = reinterpret_cast<const float2 *>(x) + sn * N + c;
#pragma unroll
      for (int t = 0; t < R; ++t) nxt[t] = sn < nsig ? p[t * R] : make_float2(0.f, 0.f);
    }
    double2 a[R];
#pragma unroll
    for (int t = 0; t < R; ++t)
      a[bit_reverse(t, LG)] = make_double2((double)cur[t].x, (double)cur[t].y);
    dft_regs<R>(a);  // a[k1] = sum_t1 z[R t1 + c] exp(-2 pi i t1 k1 / R)
#pragma unroll
    for (int k1 = 1; k1 < R; ++k1) {
      const int m = 2 * k1 * c;  // exp(-2 pi i k1 c / N) = tw[2 k1 c], or -tw[2 k1 c - N]
      const double2 w = m <= N ? tw[m] : tw[m - N];
      const double2 v = cmul(w, a[k1]);
      a[k1] = m <= N ? v : make_double2(-v.x, -v.y);
    }
    double re[R];
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) rows[k1 * (R + 1) + c] = a[k1].x;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < R; ++t) re[t] = rows[c * (R + 1) + t];
    __syncthreads();
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) rows[k1 * (R + 1) + c] = a[k1].y;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < R; ++t) a[bit_reverse(t, LG)] = make_double2(re[t], rows[c * (R + 1) + t]);
    __syncthreads();  // the rows are read out before the next signals write them
    dft_regs<R>(a);  // a[k2] = Z_{c + R k2}
    const bool valid = s < nsig;
    float *o = out + s * d;
    const int partner = g * R + ((R - c) & (R - 1));
#pragma unroll
    for (int k2 = 0; k2 < R; ++k2) {
      // Z_{n-j} for j = c + R k2: lane R - c, register R - 1 - k2; lane 0: register (R - k2) mod R
      const double2 q = a[R - 1 - k2];
      const double2 p = make_double2(__shfl(q.x, partner), __shfl(q.y, partner));
      const double2 B = c == 0 ? a[(R - k2) & (R - 1)] : p;
      const int j = c + R * k2;
      if (valid && j < d) o[j] = unpack_mag(a[k2], B, tw[j]);
    }
    if (valid && c == 0 && d > N) o[N] = unpack_mag(a[0], a[0], tw[N]);
#pragma unroll
    for (int t = 0; t < R; ++t) cur[t] = nxt[t];
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
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int cus = std::max(num_cu, 1);
  const int64_t grid = std::min<int64_t>(nsig, (int64_t)cus * per_cu);
  if (n == 64 || n == 256) {
    // four-step kernel: 64 / R signals per wave, grid capped at the blocks
    // the compute units hold at once (LDS-bound)
    const int R = n == 64 ? 8 : 16;
    const uint32_t sq_lds = R == 8 ? fft_sq_lds_bytes<8>() : fft_sq_lds_bytes<16>();
    const int sq_per_cu = std::max(1, std::min<int>(kFftBlocksPerCu, kLdsPerCu / (int)sq_lds));
    const int64_t groups = (nsig + 64 / R - 1) / (64 / R);
    const int64_t sq_grid = std::min<int64_t>(groups, (int64_t)cus * sq_per_cu);
    if (R == 8)
      HIPCHK(launch_kernel(k_fft_magnitude_sq<8>, dim3((unsigned)sq_grid), dim3(64), sq_lds, st,
                           signals, nsig, (int)d, out));
    else
      HIPCHK(launch_kernel(k_fft_magnitude_sq<16>, dim3((unsigned)sq_grid), dim3(64), sq_lds, st,
                           signals, nsig, (int)d, out));
    return HLOC_OK;
  }
  int log2n = 0;
  while ((1 << log2n) < n) ++log2n;
  HIPCHK(launch_kernel(k_fft_magnitude, dim3((unsigned)grid), dim3(64), lds,
                       st, signals, nsig, (int)len, log2n,
                       (int)d, out));
  return HLOC_OK;
}
