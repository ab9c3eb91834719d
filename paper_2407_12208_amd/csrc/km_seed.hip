// km_seed.hip -- k-means++ seeding by D^2 weighting (Arthur and Vassilvitskii;
// the paper's introduction names it as the seeding that combines with the
// mixed-precision Lloyd iteration).
//
// Centre 0 is point floor(u_0 n).  For centre i >= 1 every point's weight
// w_p = min over the chosen centres of ||x_p - c||^2 (FP64, coordinates in
// index order) is brought up to date with the newest centre, and the next
// centre is the first point p whose running sum of weights (in point order)
// exceeds u_i * sum(w).  The uniforms u_i in [0, 1) are the caller's.
// Sums are FP64 in a fixed order: per 1024-point block (each thread's four
// points in order, a fixed butterfly over the wave, the four waves in
// order), then the blocks in order, then the points of the selected block in
// order -- so the choice depends only on the data and the uniforms.
#include "km_device.hpp"
#include "km_internal.hpp"

namespace km {

constexpr int kSeedBlock = 1024;  // points per weight block (4 per thread)

// w <- min(w, ||x - c||^2) for the points of one block (w <- ||x - c||^2 on
// the first centre); bsum[block] <- sum of the block's weights.
__global__ void __launch_bounds__(256)
k_seed_update(const float* __restrict__ X, int64_t n, int d, const float* __restrict__ c, double* __restrict__ w,
              double* __restrict__ bsum, int first) {
  __shared__ float s_c[1024];
  __shared__ double s_w[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int l = tid; l < d && l < 1024; l += 256) s_c[l] = as_global(c)[l];
  __syncthreads();
  const int64_t p0 = (int64_t)blockIdx.x * kSeedBlock;
  double part = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t p = p0 + tid * 4 + q;
    if (p >= n) break;
    const KM_GLOBAL float* x = as_global(X) + p * d;
    double s = 0.0;
    for (int l = 0; l < d; ++l) {
      const double e = (double)x[l] - (double)s_c[l];
      s = __builtin_fma(e, e, s);
    }
    const double v = first ? s : __builtin_fmin(as_global(w)[p], s);
    as_global(w)[p] = v;
    part += v;
  }
  part = wave_sum(part);
  if (lane == 0) s_w[wave] = part;
  __syncthreads();
  if (tid == 0) as_global(bsum)[blockIdx.x] = ((s_w[0] + s_w[1]) + s_w[2]) + s_w[3];
}

// The next centre (one workgroup): the total, the block whose running sum
// exceeds u * total, the point inside it; its row is copied to C_row.
__global__ void __launch_bounds__(256)
k_seed_pick(const float* __restrict__ X, int64_t n, int d, const double* __restrict__ w,
            const double* __restrict__ bsum, int nblocks, double u, float* __restrict__ C_row,
            int32_t* __restrict__ idx_out, int32_t* __restrict__ pick) {
  __shared__ double s_t[256];
  __shared__ int64_t s_idx;
  const int tid = threadIdx.x;
  double t = 0.0;
  for (int b = tid; b < nblocks; b += 256) t += as_global(bsum)[b];
  s_t[tid] = t;
  __syncthreads();
  for (int o = 128; o >= 1; o >>= 1) {
    if (tid < o) s_t[tid] += s_t[tid + o];
    __syncthreads();
  }
  if (tid == 0) {
    const double total = s_t[0];
    int64_t idx = -1;
    if (total > 0.0) {
      const double target = u * total;
      double run = 0.0;
      int b = 0;
      for (; b < nblocks - 1; ++b) {
        const double nxt = run + as_global(bsum)[b];
        if (nxt > target) break;
        run = nxt;
      }
      const int64_t q0 = (int64_t)b * kSeedBlock;
      const int64_t q1 = (q0 + kSeedBlock) < n ? (q0 + kSeedBlock) : n;
      int64_t last = -1;
      for (int64_t p = q0; p < q1; ++p) {
        const double wp = as_global(w)[p];
        if (wp > 0.0) last = p;
        run += wp;
        if (run > target && wp > 0.0) {
          idx = p;
          break;
        }
      }
      if (idx < 0) idx = last;  // rounding left the target past the block's last weight
    }
    if (idx < 0) {  // every weight zero: the points coincide with the centres
      idx = (int64_t)(u * (double)n);
      if (idx >= n) idx = n - 1;
    }
    s_idx = idx;
    if (idx_out) *as_global(idx_out) = (int32_t)idx;
    *as_global(pick) = (int32_t)idx;
  }
  __syncthreads();
  const int64_t idx = s_idx;
  for (int l = tid; l < d; l += 256) as_global(C_row)[l] = as_global(X)[idx * d + l];
}

// first centre: point floor(u n)
__global__ void k_seed_first(const float* __restrict__ X, int64_t n, int d, double u, float* __restrict__ C_row,
                             int32_t* __restrict__ idx_out) {
  int64_t idx = (int64_t)(u * (double)n);
  if (idx >= n) idx = n - 1;
  for (int l = threadIdx.x; l < d; l += blockDim.x) as_global(C_row)[l] = as_global(X)[idx * d + l];
  if (threadIdx.x == 0 && idx_out) *as_global(idx_out) = (int32_t)idx;
}

hipError_t launch_seed_pp(const float* X, int64_t n, int d, int k, const double* u, float* C, int32_t* idx,
                          double* w, double* bsum, int32_t* pick, hipStream_t st) {
  const int nblocks = (int)((n + kSeedBlock - 1) / kSeedBlock);
  hipLaunchKernelGGL(k_seed_first, dim3(1), dim3(256), 0, st, X, n, d, u[0], C, idx);
  for (int i = 1; i < k; ++i) {
    hipLaunchKernelGGL(k_seed_update, dim3(nblocks), dim3(256), 0, st, X, n, d, C + (int64_t)(i - 1) * d, w,
                       bsum, i == 1 ? 1 : 0);
    hipLaunchKernelGGL(k_seed_pick, dim3(1), dim3(256), 0, st, X, n, d, w, bsum, nblocks, u[i],
                       C + (int64_t)i * d, idx ? idx + i : nullptr, pick);
  }
  return hipGetLastError();
}

}  // namespace km
