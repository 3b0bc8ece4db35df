// Database set-up kernels: region-contiguous re-layout of the rows, FP64 row
// norms, region representatives (mean of the member rows, accumulated in
// FP64), their fp32 copies and norms, and the tile of each floor-plan
// position (Section 3.2: floor(coord / cell) in FP64 from origin (0, 0)).
#include "hloc_device.h"
#include "hloc_internal.h"

namespace hloc {

// dst row i (stride dp, zero padded) = src row src_row[i] (first d values).
__global__ void k_gather_rows(const float *__restrict__ src, const int32_t *__restrict__ src_row,
                              int64_t n, int d, int src_stride, float *__restrict__ dst, int dp) {
  const int64_t i = blockIdx.x * 4 + wave_id();
  if (i >= n) return;
  const float *s = src + (int64_t)src_row[i] * src_stride;
  float *o = dst + i * dp;
  for (int c = lane_id(); c < dp; c += 64) o[c] = c < d ? s[c] : 0.f;
}

hipError_t launch_gather_rows(const float *src, const int32_t *src_row, int64_t n, int32_t d,
                              int32_t src_stride, float *dst, int32_t dp, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  return launch_kernel(k_gather_rows, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, src, src_row,
                     n, d, src_stride, dst, dp);
}

// Squared norm of each row summed in FP64, stored rounded to fp32; the
// largest norm goes to *max_norm (non-negative floats order like their bits).
constexpr int kNormRowsPerWave = 16;

// FP64 squared norm of each row (stored as fp32), kNormRowsPerWave rows per
// wave; the largest norm goes to *max_norm with one atomic per block.
__global__ void k_row_norms(const float *__restrict__ rows, int64_t n, int dp, float *n2,
                            float *max_norm) {
  __shared__ float s_m[4];
  const int64_t i0 = ((int64_t)blockIdx.x * 4 + wave_id()) * kNormRowsPerWave;
  float m = 0.f;
  for (int64_t i = i0; i < min(n, i0 + kNormRowsPerWave); ++i) {
    const float *r = rows + i * dp;
    double acc = 0.0;
    for (int c = lane_id(); c < dp; c += 64) acc = fma((double)r[c], (double)r[c], acc);
    acc = wave_sum_f64(acc);
    if (lane_id() == 0) n2[i] = (float)acc;
    m = fmaxf(m, (float)sqrt(acc));
  }
  if (lane_id() == 0) s_m[wave_id()] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicMax(reinterpret_cast<unsigned int *>(max_norm),
              __float_as_uint(fmaxf(fmaxf(s_m[0], s_m[1]), fmaxf(s_m[2], s_m[3]))));
}

hipError_t launch_row_norms(const float *rows, int64_t n, int32_t dp, float *n2,
                            float *max_norm, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t per_block = 4 * kNormRowsPerWave;
  return launch_kernel(k_row_norms, dim3((unsigned)((n + per_block - 1) / per_block)), dim3(256),
                       0, s, rows, n, dp, n2, max_norm);
}

// Mean of each region's rows: one block per region, threads over columns,
// rows summed in order in FP64.
__global__ void k_region_means(const float *__restrict__ rows,
                               const int64_t *__restrict__ reg_start, int R, int dp,
                               double *__restrict__ mean64) {
  const int r = blockIdx.x;
  if (r >= R) return;
  const int64_t b = reg_start[r], e = reg_start[r + 1];
  for (int c = threadIdx.x; c < dp; c += blockDim.x) {
    double acc = 0.0;
    for (int64_t i = b; i < e; ++i) acc += (double)rows[i * dp + c];
    mean64[(int64_t)r * dp + c] = e > b ? acc / (double)(e - b) : 0.0;
  }
}

hipError_t launch_region_means(const float *rows, const int64_t *reg_start, int32_t R,
                               int32_t dp, double *mean64, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  return launch_kernel(k_region_means, dim3(R), dim3(256), 0, s, rows, reg_start, R, dp, mean64);
}

// fp32 copy and FP64 squared norm (stored as fp32) of each representative;
// empty regions get norm +inf so that the screen never selects them.
__global__ void k_rep_finish(const double *__restrict__ rep64,
                             const int64_t *__restrict__ reg_start, int R, int dp,
                             float *__restrict__ rep32, float *__restrict__ rep_n2,
                             float *max_norm) {
  const int r = blockIdx.x * 4 + wave_id();
  if (r >= R) return;
  const bool empty = reg_start[r + 1] == reg_start[r];
  const double *src = rep64 + (int64_t)r * dp;
  float *dst = rep32 + (int64_t)r * dp;
  double acc = 0.0;
  for (int c = lane_id(); c < dp; c += 64) {
    const double v = empty ? 0.0 : src[c];
    dst[c] = (float)v;
    acc = fma(v, v, acc);
  }
  acc = wave_sum_f64(acc);
  if (lane_id() == 0) {
    rep_n2[r] = empty ? __builtin_inff() : (float)acc;
    if (!empty)
      atomicMax(reinterpret_cast<unsigned int *>(max_norm), __float_as_uint((float)sqrt(acc)));
  }
}

hipError_t launch_rep_finish(const double *rep64, const int64_t *reg_start, int32_t R,
                             int32_t dp, float *rep32, float *rep_n2, float *max_norm,
                             hipStream_t s) {
  if (R <= 0) return hipSuccess;
  return launch_kernel(k_rep_finish, dim3((R + 3) / 4), dim3(256), 0, s, rep64, reg_start, R, dp,
                     rep32, rep_n2, max_norm);
}

__global__ void k_tiles(const double *__restrict__ xy, int64_t n, double cell,
                        int2 *__restrict__ tile) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double tx = floor(__ddiv_rn(xy[2 * i], cell));
  const double ty = floor(__ddiv_rn(xy[2 * i + 1], cell));
  tile[i] = make_int2((int)tx, (int)ty);
}

hipError_t launch_tiles(const double *xy, int64_t n, double cell, int2 *tile, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  return launch_kernel(k_tiles, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, xy, n, cell,
                     tile);
}

}  // namespace hloc
